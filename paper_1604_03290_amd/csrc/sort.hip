// Stable least-significant-digit radix sort of (uint64 key, int32 value) pairs, 8-bit
// digits, one pass per digit.  Each pass:
//   histogram  per tile of 4096 items (256 threads x 16 rounds), the digit counts in
//              LDS, stored digit-major: hist[d * tiles + tile]
//   scan       exclusive scan of hist: where digit d of each tile starts in the output
//   scatter    the tile again, in its order (round, then wavefront, then lane): each
//              item's destination is its tile's start for the digit plus the items of
//              that digit before it in the tile, found by the wavefront's ballots
//              (lanes with the same digit), the counts of the earlier wavefronts of
//              the round and a running count per digit over the rounds
// Equal keys keep their input order, so the sort is stable.
#include "common.hpp"

namespace sph {
namespace {

constexpr int kDigitBits = 8;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kRounds = 16;
constexpr int kSortTile = kBlock * kRounds;
constexpr int kWaves = kBlock / 64;

__device__ inline int digit_of(uint64_t key, int shift) { return (int)((key >> shift) & (kDigits - 1)); }

__global__ __launch_bounds__(kBlock) void k_digit_hist(const uint64_t *__restrict__ key, int64_t n,
                                                       int shift, int32_t *__restrict__ hist,
                                                       int64_t tiles) {
    __shared__ int32_t cnt[kDigits];
    cnt[threadIdx.x] = 0;  // kBlock == kDigits
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[digit_of(key[i], shift)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_digit_scatter(const uint64_t *__restrict__ kin,
                                                          const int32_t *__restrict__ vin,
                                                          int64_t n, int shift,
                                                          const int32_t *__restrict__ start,
                                                          int64_t tiles,
                                                          uint64_t *__restrict__ kout,
                                                          int32_t *__restrict__ vout) {
    __shared__ int32_t run[kDigits];             // next output position of each digit
    __shared__ int32_t wcnt[kWaves][kDigits];    // this round's count per wavefront
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    run[t] = start[(int64_t)t * tiles + blockIdx.x];
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;  // lanes below this one
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kRounds; ++r) {
#pragma unroll
        for (int q = 0; q < kWaves; ++q) wcnt[q][t] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)r * kBlock + t;
        const bool valid = i < n;
        const uint64_t k = valid ? kin[i] : 0;
        const int d = digit_of(k, shift);
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kDigitBits; ++b) {
            const uint64_t ones = __ballot((d >> b) & 1);
            same &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int below = __popcll(same & lt);
        if (valid && below == 0) wcnt[w][d] = __popcll(same);  // the digit's lowest lane
        __syncthreads();
        int before = 0;
        for (int q = 0; q < w; ++q) before += wcnt[q][d];
        if (valid) {
            const int dst = run[d] + before + below;
            kout[dst] = k;
            vout[dst] = vin[i];
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) add += wcnt[q][t];
        run[t] += add;
        // the next round's clearing of wcnt follows a barrier after these reads
        __syncthreads();
    }
}

}  // namespace

// Scratch elements (int32) of radix_sort_pairs for n items.
size_t radix_sort_tmp_elems(int64_t n) {
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t m = tiles * kDigits;
    return (size_t)(m + 1) + scan_tmp_elems(m + 1) + 64;
}

// Sorts (key[0], val[0]) by bits [0, bits) of the keys; the result is in buffer
// *which (0 or 1) of the double buffers.  tmp: radix_sort_tmp_elems(n) int32.
int radix_sort_pairs(uint64_t *key[2], int32_t *val[2], int64_t n, int bits, int32_t *tmp,
                     int *which, hipStream_t s) {
    *which = 0;
    if (n <= 1) return SPH_OK;
    if (n >= ((int64_t)1 << 31)) return fail(SPH_ERR_INVALID_ARG, "radix sort of 2^31 items or more");
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t m = tiles * kDigits;
    int32_t *hist = tmp;
    int32_t *scan = tmp + m + 1;
    int cur = 0;
    for (int shift = 0; shift < bits; shift += kDigitBits) {
        k_digit_hist<<<(unsigned)tiles, kBlock, 0, s>>>(key[cur], n, shift, hist, tiles);
        SPH_LAUNCHED();
        int rc = exclusive_scan_i32(hist, hist, m, scan, s);
        if (rc) return rc;
        k_digit_scatter<<<(unsigned)tiles, kBlock, 0, s>>>(key[cur], val[cur], n, shift, hist, tiles,
                                                            key[cur ^ 1], val[cur ^ 1]);
        SPH_LAUNCHED();
        cur ^= 1;
    }
    *which = cur;
    return SPH_OK;
}

}  // namespace sph
