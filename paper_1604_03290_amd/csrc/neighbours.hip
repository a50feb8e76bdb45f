// Interaction partner lists (section 3.5.2) as a CSR in user order, each row
// ascending.  Positions are first gathered into slot order; the count and fill
// passes take candidates from the grid's pair list when it has one (else from
// the cell rows) and apply the exact test; each row is then sorted by one
// wavefront with a bitonic network in LDS.
#include <climits>

#include "common.hpp"
#include "rhs_common.hpp"

namespace sph {
namespace {

constexpr int kSortMax = 1024;  // longest row sorted in LDS by one wavefront

__global__ __launch_bounds__(kBlock) void k_nb_gather(GridDev g, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, int64_t n,
                                                      double4 *__restrict__ pos,
                                                      int32_t *__restrict__ status) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = g.perm[s];
    const double px = x[a], py = y[a], pz = z[a];
    if (!within_cell(g, (int)s, px, py, pz)) raise_flag(status, SPH_ERR_STALE_GRID);
    if (!(isfinite(px) && isfinite(py) && isfinite(pz))) raise_flag(status, SPH_ERR_DOMAIN);
    pos[s] = make_double4(px, py, pz, 0.0);
}

template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_nb_pass(GridDev g, const double4 *__restrict__ pos,
                                                    int64_t n, double h2, double reach,
                                                    int64_t *__restrict__ count,
                                                    const int64_t *__restrict__ row_ptr,
                                                    int32_t *__restrict__ col) {
    const int64_t s = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (s >= n) return;
    const double4 pa = pos[s];
    const int a = g.perm[s];
    int64_t k = kFill ? row_ptr[a] : 0;
    for_each_candidate(g, s, pa.x, pa.y, pa.z, reach, [&](int t) {
        const double4 pb = pos[t];
        if (dist2_exact(pa.x, pa.y, pa.z, pb.x, pb.y, pb.z) < h2) {
            if (kFill) col[k] = g.perm[t];
            ++k;
        }
    });
    if (!kFill) count[a] = k;
}

// one wavefront per row: bitonic sort of the row in LDS (rows longer than
// kSortMax, which no workload here produces, fall back to an insertion sort)
__global__ __launch_bounds__(kBlock) void k_nb_sort(const int64_t *__restrict__ row_ptr,
                                                    int64_t n, int32_t *__restrict__ col) {
    __shared__ int32_t lds[kBlock / 64][kSortMax];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t *buf = lds[wave];
    const int64_t a = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    if (a >= n) return;
    const int64_t r0 = row_ptr[a];
    const int len = (int)(row_ptr[a + 1] - r0);
    if (len <= 1) return;
    if (len > kSortMax) {
        if (lane == 0) {
            for (int64_t i = r0 + 1; i < r0 + len; ++i) {
                const int32_t v = col[i];
                int64_t j = i - 1;
                while (j >= r0 && col[j] > v) {
                    col[j + 1] = col[j];
                    --j;
                }
                col[j + 1] = v;
            }
        }
        return;
    }
    int n2 = 2;
    while (n2 < len) n2 <<= 1;
    for (int i = lane; i < n2; i += 64) buf[i] = i < len ? col[r0 + i] : INT_MAX;
    wave_sync();
    for (int kk = 2; kk <= n2; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < n2; i += 64) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const int32_t u = buf[i], v = buf[ixj];
                    const bool up = (i & kk) == 0;
                    if ((u > v) == up) {
                        buf[i] = v;
                        buf[ixj] = u;
                    }
                }
            }
            wave_sync();
        }
    }
    for (int i = lane; i < len; i += 64) col[r0 + i] = buf[i];
}

}  // namespace

size_t neighbours_ws_bytes(int64_t n) {
    Carve c(nullptr);
    c.take<double4>(n);
    c.take<int64_t>(n);
    c.take<int64_t>(scan_tmp_elems(n));
    return c.used;
}

}  // namespace sph

using namespace sph;

extern "C" int sph_neighbours(const sph_grid *grid, const double *x, const double *y,
                              const double *z, double h, int64_t *row_ptr, int32_t *col,
                              int64_t col_cap, int64_t *nnz_out, void *ws, size_t ws_bytes,
                              void *stream) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!x || !y || !z || !row_ptr || !nnz_out || !ws || (!col && col_cap > 0))
        return fail(SPH_ERR_INVALID_ARG, "null pointer");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(SPH_ERR_INVALID_ARG, "h must be positive");
    if (h > grid->h) return fail(SPH_ERR_INVALID_ARG, "h exceeds the grid's support radius");
    const int64_t n = grid->n;
    const size_t need = neighbours_ws_bytes(n);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    Carve c(ws);
    double4 *pos = c.take<double4>(n);
    int64_t *count = c.take<int64_t>(n);
    int64_t *tmp = c.take<int64_t>(scan_tmp_elems(n));
    GridDev g = grid_dev(grid);
    const double reach = (h + g.delta) * (1.0 + 1e-9);
    if ((rc = clear_status(ws, s))) return rc;
    k_nb_gather<<<blocks_for(n), kBlock, 0, s>>>(g, x, y, z, n, pos, c.status());
    SPH_LAUNCHED();
    k_nb_pass<false><<<blocks_for(n), kBlock, 0, s>>>(g, pos, n, h * h, reach, count, nullptr, nullptr);
    SPH_LAUNCHED();
    if ((rc = exclusive_scan_i64(count, row_ptr, n, tmp, s))) return rc;
    int64_t nnz = 0;
    int32_t flag = 0;
    SPH_HIP_TRY(hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPH_HIP_TRY(hipMemcpyAsync(&flag, c.status(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPH_HIP_TRY(hipStreamSynchronize(s));
    *nnz_out = nnz;
    if (flag) return fail(flag, "device flag %d raised while counting partners", flag);
    if (nnz > col_cap)
        return fail(SPH_ERR_CAPACITY, "%lld partners exceed capacity %lld", (long long)nnz,
                    (long long)col_cap);
    k_nb_pass<true><<<blocks_for(n), kBlock, 0, s>>>(g, pos, n, h * h, reach, nullptr, row_ptr, col);
    SPH_LAUNCHED();
    k_nb_sort<<<blocks_for(n, kBlock / 64), kBlock, 0, s>>>(row_ptr, n, col);
    SPH_LAUNCHED();
    return SPH_OK;
}
