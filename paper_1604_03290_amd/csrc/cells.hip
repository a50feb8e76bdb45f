// Cell list ("helping grid" of section 3.5.2): bin, count, scan, scatter, and
// order every cell by user index.  The slot order is a counting sort on the
// cell number (one radix digit of size ncells; cells numbered by tiles and blocks,
// see common.hpp) made deterministic by the per-cell ordering, so repeated builds
// give identical permutations.
#include <cfloat>

#include "common.hpp"

namespace sph {
namespace {

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_bin(const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z, int64_t n,
                                                GridDev g, int32_t *__restrict__ key,
                                                int32_t *__restrict__ count,
                                                int32_t *__restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double px = x[i], py = y[i], pz = z[i];
    if (!(isfinite(px) && isfinite(py) && isfinite(pz))) raise_flag(status, SPH_ERR_DOMAIN);
    const int ix = cell_index(px, g.lox, g.inv_cell, g.nx);
    const int iy = cell_index(py, g.loy, g.inv_cell, g.ny);
    const int iz = cell_index(pz, g.loz, g.inv_cell, g.nz);
    const int c = cell_number(ix, iy, iz, g.nbx, g.nby);
    key[i] = c;
    atomicAdd(&count[c], 1);
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t *__restrict__ key, int64_t n,
                                                    const int32_t *__restrict__ start,
                                                    int32_t *__restrict__ cursor,
                                                    int32_t *__restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = key[i];
    const int slot = start[c] + atomicAdd(&cursor[c], 1);
    perm[slot] = (int32_t)i;
}

// one thread per cell: insertion sort of its slots by user index (cells hold
// tens of particles), then record each slot's cell
__global__ __launch_bounds__(kBlock) void k_order_cells(const int32_t *__restrict__ start,
                                                        int64_t ncells,
                                                        int32_t *__restrict__ perm,
                                                        int32_t *__restrict__ cell_of) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int s0 = start[c], s1 = start[c + 1];
    for (int i = s0 + 1; i < s1; ++i) {
        const int v = perm[i];
        int j = i - 1;
        while (j >= s0 && perm[j] > v) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
    for (int i = s0; i < s1; ++i) cell_of[i] = (int32_t)c;
}

// the status flag and the header's second word (sph_neighbours' moved flag)
__global__ void k_clear_status(int32_t *status) {
    status[0] = 0;
    status[1] = 0;
}

}  // namespace

int clear_status(void *ws, hipStream_t s) {
    k_clear_status<<<1, 1, 0, s>>>((int32_t *)ws);
    SPH_LAUNCHED();
    return SPH_OK;
}

size_t build_ws_bytes(int64_t n, int64_t ncells);

int check_grid(const sph_grid *g) {
    if (!g) return fail(SPH_ERR_INVALID_ARG, "grid is NULL");
    if (!g->perm || !g->cell_start || !g->cell_of)
        return fail(SPH_ERR_INVALID_ARG, "grid arrays are NULL");
    if (g->n <= 0 || g->dims[0] <= 0 || g->dims[1] <= 0 || g->dims[2] <= 0 ||
        !(g->cell > 0.0) || !(g->h > 0.0) || !(g->skin >= 0.0) ||
        g->ncells != (int64_t)kBlockCells * blocks_along(g->dims[0]) * blocks_along(g->dims[1]) *
                         blocks_along(g->dims[2]))
        return fail(SPH_ERR_INVALID_ARG, "grid is not initialised");
    return SPH_OK;
}

}  // namespace sph

using namespace sph;

extern "C" int sph_grid_geometry(const double lo[3], const double hi[3], double h, double skin,
                                 int cells_per_h, int32_t dims_out[3], int64_t *ncells_out,
                                 double *cell_out) {
    clear_error();
    if (!lo || !hi || !dims_out || !ncells_out || !cell_out)
        return fail(SPH_ERR_INVALID_ARG, "null pointer");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(SPH_ERR_INVALID_ARG, "h must be positive");
    if (!(skin >= 0.0) || !std::isfinite(skin))
        return fail(SPH_ERR_INVALID_ARG, "skin must be >= 0");
    if (cells_per_h != 1 && cells_per_h != 2)
        return fail(SPH_ERR_INVALID_ARG, "cells_per_h must be 1 or 2");
    const double cell = (h + skin) * (1.0 + 0x1p-40) / cells_per_h;
    int64_t total = kBlockCells;
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(hi[d] > lo[d]))
            return fail(SPH_ERR_INVALID_ARG, "box must satisfy lo < hi (axis %d)", d);
        const double cnt = std::ceil((hi[d] - lo[d]) / cell);
        if (cnt > 1.0e6) return fail(SPH_ERR_INVALID_ARG, "more than 1e6 cells along axis %d", d);
        dims_out[d] = cnt < 1.0 ? 1 : (int32_t)cnt;
        total *= blocks_along(dims_out[d]);
    }
    if (total >= ((int64_t)1 << 31) - 1) return fail(SPH_ERR_INVALID_ARG, "too many cells");
    *ncells_out = total;
    *cell_out = cell;
    return SPH_OK;
}

size_t sph::build_ws_bytes(int64_t n, int64_t ncells) {
    Carve c(nullptr);
    c.take<int32_t>(n);                    // key
    c.take<int32_t>(ncells);               // cursor
    c.take<int32_t>(scan_tmp_elems(ncells));  // scan tiles
    return c.used;
}

extern "C" int sph_build_cells(const double *x, const double *y, const double *z, int64_t n,
                               const double lo[3], const double hi[3], double h, double skin,
                               int cells_per_h, int32_t *perm, int32_t *cell_start,
                               int64_t ncells_cap, int32_t *cell_of, sph_grid *grid_out,
                               void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!x || !y || !z || !perm || !cell_start || !cell_of || !grid_out || !ws)
        return fail(SPH_ERR_INVALID_ARG, "null pointer");
    if (n <= 0 || n >= ((int64_t)1 << 31) - 1)
        return fail(SPH_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1)");
    int32_t dims[3];
    int64_t ncells;
    double cell;
    int rc = sph_grid_geometry(lo, hi, h, skin, cells_per_h, dims, &ncells, &cell);
    if (rc) return rc;
    grid_out->n = n;
    for (int d = 0; d < 3; ++d) {
        grid_out->dims[d] = dims[d];
        grid_out->lo[d] = lo[d];
    }
    grid_out->ncells = ncells;
    grid_out->cell = cell;
    grid_out->h = h;
    grid_out->skin = skin;
    grid_out->perm = perm;
    grid_out->cell_start = cell_start;
    grid_out->cell_of = cell_of;
    grid_out->pairs = nullptr;
    if (ncells > ncells_cap)
        return fail(SPH_ERR_CAPACITY, "grid needs %lld cells, capacity %lld", (long long)ncells,
                    (long long)ncells_cap);
    const size_t need = build_ws_bytes(n, ncells);
    if (ws_bytes < need)
        return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);

    hipStream_t s = (hipStream_t)stream;
    Carve c(ws);
    int32_t *key = c.take<int32_t>(n);
    int32_t *cursor = c.take<int32_t>(ncells);
    int32_t *tmp = c.take<int32_t>(scan_tmp_elems(ncells));
    GridDev g = grid_dev(grid_out);

    if ((rc = clear_status(ws, s))) return rc;
    k_fill_i32<<<blocks_for(ncells + 1), kBlock, 0, s>>>(cell_start, ncells + 1, 0);
    SPH_LAUNCHED();
    k_fill_i32<<<blocks_for(ncells), kBlock, 0, s>>>(cursor, ncells, 0);
    SPH_LAUNCHED();
    k_bin<<<blocks_for(n), kBlock, 0, s>>>(x, y, z, n, g, key, cell_start, c.status());
    SPH_LAUNCHED();
    if ((rc = exclusive_scan_i32(cell_start, cell_start, ncells, tmp, s))) return rc;
    k_scatter<<<blocks_for(n), kBlock, 0, s>>>(key, n, cell_start, cursor, perm);
    SPH_LAUNCHED();
    k_order_cells<<<blocks_for(ncells), kBlock, 0, s>>>(cell_start, ncells, perm, cell_of);
    SPH_LAUNCHED();
    return SPH_OK;
}
