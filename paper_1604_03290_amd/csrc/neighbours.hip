// Interaction partner lists (section 3.5.2) as a CSR in user order, each row
// ascending.  Count pass -> scan -> fill pass -> per-row ordering.
#include "common.hpp"

namespace sph {
namespace {

struct Pos {
    const double *__restrict__ x;
    const double *__restrict__ y;
    const double *__restrict__ z;
};

__global__ __launch_bounds__(kBlock) void k_nb_count(GridDev g, Pos p, int64_t n, double h2,
                                                     double reach, int64_t *__restrict__ count,
                                                     int32_t *__restrict__ status) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = g.perm[s];
    const double xa = p.x[a], ya = p.y[a], za = p.z[a];
    if (!within_cell(g, (int)s, xa, ya, za)) raise_flag(status, SPH_ERR_STALE_GRID);
    int64_t c = 0;
    for_each_row(g, xa, ya, za, reach, [&](int s0, int s1) {
        for (int t = s0; t < s1; ++t) {
            if (t == s) continue;
            const int b = g.perm[t];
            c += dist2_exact(xa, ya, za, p.x[b], p.y[b], p.z[b]) < h2;
        }
    });
    count[a] = c;
}

__global__ __launch_bounds__(kBlock) void k_nb_fill(GridDev g, Pos p, int64_t n, double h2,
                                                    double reach,
                                                    const int64_t *__restrict__ row_ptr,
                                                    int32_t *__restrict__ col) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = g.perm[s];
    const double xa = p.x[a], ya = p.y[a], za = p.z[a];
    int64_t k = row_ptr[a];
    for_each_row(g, xa, ya, za, reach, [&](int s0, int s1) {
        for (int t = s0; t < s1; ++t) {
            if (t == s) continue;
            const int b = g.perm[t];
            if (dist2_exact(xa, ya, za, p.x[b], p.y[b], p.z[b]) < h2) col[k++] = b;
        }
    });
}

__global__ __launch_bounds__(kBlock) void k_nb_sort(const int64_t *__restrict__ row_ptr,
                                                    int64_t n, int32_t *__restrict__ col) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int64_t r0 = row_ptr[a], r1 = row_ptr[a + 1];
    for (int64_t i = r0 + 1; i < r1; ++i) {
        const int32_t v = col[i];
        int64_t j = i - 1;
        while (j >= r0 && col[j] > v) {
            col[j + 1] = col[j];
            --j;
        }
        col[j + 1] = v;
    }
}

}  // namespace

size_t neighbours_ws_bytes(int64_t n) {
    Carve c(nullptr);
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
    int64_t *count = c.take<int64_t>(n);
    int64_t *tmp = c.take<int64_t>(scan_tmp_elems(n));
    GridDev g = grid_dev(grid);
    const Pos p{x, y, z};
    const double reach = (h + g.delta) * (1.0 + 1e-9);
    if ((rc = clear_status(ws, s))) return rc;
    k_nb_count<<<blocks_for(n), kBlock, 0, s>>>(g, p, n, h * h, reach, count, c.status());
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
    k_nb_fill<<<blocks_for(n), kBlock, 0, s>>>(g, p, n, h * h, reach, row_ptr, col);
    SPH_LAUNCHED();
    k_nb_sort<<<blocks_for(n), kBlock, 0, s>>>(row_ptr, n, col);
    SPH_LAUNCHED();
    return SPH_OK;
}
