// Exclusive prefix sums (int32 / int64) in three deterministic passes:
// per-tile totals, a scan of the tile totals by one workgroup, per-tile scan
// plus offset.  out has n + 1 entries; out[n] receives the total.  In-place
// (in == out) is allowed.
#include "common.hpp"

namespace sph {
namespace {

constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

template <class T>
__device__ T block_exclusive_scan(T v, T *lds, T *total) {
    // Hillis-Steele over the 256 thread totals in LDS
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        T add = t >= off ? lds[t - off] : T(0);
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    T incl = lds[t];
    *total = lds[kBlock - 1];
    __syncthreads();
    return incl - v;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const T *__restrict__ in, int64_t n,
                                                      T *__restrict__ sums) {
    __shared__ T lds[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) s += in[base + k];
    T total;
    block_exclusive_scan<T>(s, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_sums(T *__restrict__ sums, int64_t m) {
    __shared__ T lds[kBlock];
    T carry = 0;
    for (int64_t base = 0; base < m; base += kTile) {
        T v[kItems];
        T s = 0;
        const int64_t b = base + (int64_t)threadIdx.x * kItems;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            v[k] = (b + k < m) ? sums[b + k] : T(0);
            s += v[k];
        }
        T total;
        T ex = block_exclusive_scan<T>(s, lds, &total) + carry;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (b + k < m) sums[b + k] = ex;
            ex += v[k];
        }
        carry += total;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const T *in, T *out, int64_t n,
                                                      const T *__restrict__ sums) {
    __shared__ T lds[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : T(0);
        s += v[k];
    }
    T total;
    T ex = block_exclusive_scan<T>(s, lds, &total) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    // the last tile writes the grand total
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = ex;
}

template <class T>
int scan_impl(const T *in, T *out, int64_t n, T *tmp, hipStream_t s) {
    if (n <= 0) return SPH_OK;
    const unsigned tiles = blocks_for(n, kTile);
    k_tile_sums<T><<<tiles, kBlock, 0, s>>>(in, n, tmp);
    SPH_LAUNCHED();
    k_scan_sums<T><<<1, kBlock, 0, s>>>(tmp, (int64_t)tiles);
    SPH_LAUNCHED();
    k_tile_scan<T><<<tiles, kBlock, 0, s>>>(in, out, n, tmp);
    SPH_LAUNCHED();
    return SPH_OK;
}

}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)blocks_for(n > 0 ? n : 1, kTile); }

int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s) {
    return scan_impl<int32_t>(in, out, n, tmp, s);
}

int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, tmp, s);
}

}  // namespace sph
