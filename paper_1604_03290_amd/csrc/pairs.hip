// Frozen candidate-pair list ("interactionsList" of section 3.5.2 with a
// skin): for every slot, the slots whose distance was below h + skin when the
// list was built.  While every particle stays within skin/2 of its position at
// build time this is a superset of its partners, and the pair kernels re-test
// d^2 < h^2 exactly at the current positions.
//
// Layout: slots are grouped in blocks of 64 (one wavefront); inside block B the
// j-th candidate of the block's lane l sits at slot[block_start[B] + 64 j + l],
// so the j-th loads of a wavefront are contiguous.  Each block is padded to its
// longest list.
#include "common.hpp"
#include "rhs_common.hpp"

namespace sph {
namespace {

constexpr int kWave = 64;

__global__ __launch_bounds__(kBlock) void k_pl_gather(GridDev g, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, int64_t n,
                                                      double *__restrict__ x0,
                                                      int32_t *__restrict__ status) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = g.perm[s];
    const double px = x[a], py = y[a], pz = z[a];
    if (!within_cell(g, (int)s, px, py, pz)) raise_flag(status, SPH_ERR_STALE_GRID);
    x0[3 * s + 0] = px;
    x0[3 * s + 1] = py;
    x0[3 * s + 2] = pz;
}

// Count pass (kFill = false) or fill pass.  The fill runs over every slot of
// every group, including the lanes past n of the last group, and fills the
// padding after each list with the slot itself (n - 1 for lanes past n), so
// that every entry of a group is a valid slot and readers of whole groups load
// without guards.
template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_pl_scan(GridDev g, const double *__restrict__ x0,
                                                    int64_t n, double r2, double reach,
                                                    int32_t *__restrict__ count,
                                                    const int64_t *__restrict__ block_start,
                                                    int32_t *__restrict__ slot) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (n + kWave - 1) / kWave;
    if (s >= (kFill ? nb * kWave : n)) return;
    int64_t base = 0, maxc = 0;
    if (kFill) {
        base = block_start[s / kWave] + (s % kWave);
        maxc = (block_start[s / kWave + 1] - block_start[s / kWave]) / kWave;
        if (s >= n) {
            for (int64_t j = 0; j < maxc; ++j) slot[base + kWave * j] = (int32_t)(n - 1);
            return;
        }
    }
    const double xa = x0[3 * s], ya = x0[3 * s + 1], za = x0[3 * s + 2];
    int c = 0;
    for_each_row(g, xa, ya, za, reach, [&](int s0, int s1) {
        for (int t = s0; t < s1; ++t) {
            if (t == s) continue;
            if (dist2_exact(xa, ya, za, x0[3 * t], x0[3 * t + 1], x0[3 * t + 2]) < r2) {
                if (kFill) slot[base + (int64_t)kWave * c] = t;
                ++c;
            }
        }
    });
    if (kFill)
        for (int64_t j = c; j < maxc; ++j) slot[base + kWave * j] = (int32_t)s;
    else
        count[s] = c;
}

// sizes[B] = 64 * (longest list of block B)
__global__ __launch_bounds__(kBlock) void k_pl_sizes(const int32_t *__restrict__ count, int64_t n,
                                                     int64_t *__restrict__ sizes) {
    const int64_t B = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (n + kWave - 1) / kWave;
    if (B >= nb) return;
    int m = 0;
    for (int64_t s = B * kWave; s < min((B + 1) * kWave, n); ++s) m = max(m, count[s]);
    sizes[B] = (int64_t)kWave * m;
}

}  // namespace

size_t pairs_ws_bytes(int64_t n) {
    Carve c(nullptr);
    const int64_t nb = (n + kWave - 1) / kWave;
    c.take<int64_t>(nb);
    c.take<int64_t>(scan_tmp_elems(nb));
    return c.used;
}

}  // namespace sph

using namespace sph;

extern "C" int sph_build_pairs(sph_grid *grid, const double *x, const double *y, const double *z,
                               sph_pairs *out, int32_t *count, int64_t *block_start,
                               int32_t *slot, int64_t capacity, double *x0, int64_t *needed,
                               void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!x || !y || !z || !out || !count || !block_start || !x0 || !needed || !ws ||
        (!slot && capacity > 0))
        return fail(SPH_ERR_INVALID_ARG, "null pointer");
    const int64_t n = grid->n;
    const size_t need = pairs_ws_bytes(n);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    Carve c(ws);
    const int64_t nb = (n + 63) / 64;
    int64_t *sizes = c.take<int64_t>(nb);
    int64_t *tmp = c.take<int64_t>(scan_tmp_elems(nb));
    GridDev g = grid_dev(grid);
    g.pl_count = nullptr;  // the cells, not a previous list, locate the candidates
    g.pl_block = nullptr;
    g.pl_slot = nullptr;
    g.pl_x0 = nullptr;
    const double radius = grid->h + grid->skin;
    const double r2 = radius * radius * (1.0 + 1e-12);
    const double reach = (radius + g.delta) * (1.0 + 1e-9);
    if ((rc = clear_status(ws, s))) return rc;
    k_pl_gather<<<blocks_for(n), kBlock, 0, s>>>(g, x, y, z, n, x0, c.status());
    SPH_LAUNCHED();
    k_pl_scan<false><<<blocks_for(n), kBlock, 0, s>>>(g, x0, n, r2, reach, count, nullptr, nullptr);
    SPH_LAUNCHED();
    k_pl_sizes<<<blocks_for(nb), kBlock, 0, s>>>(count, n, sizes);
    SPH_LAUNCHED();
    if ((rc = exclusive_scan_i64(sizes, block_start, nb, tmp, s))) return rc;
    int64_t total = 0;
    int32_t flag = 0;
    SPH_HIP_TRY(hipMemcpyAsync(&total, block_start + nb, sizeof total, hipMemcpyDeviceToHost, s));
    SPH_HIP_TRY(hipMemcpyAsync(&flag, c.status(), sizeof flag, hipMemcpyDeviceToHost, s));
    SPH_HIP_TRY(hipStreamSynchronize(s));
    *needed = total;
    if (flag) return fail(flag, "device flag %d raised while building the pair list", flag);
    if (total > capacity)
        return fail(SPH_ERR_CAPACITY, "pair list needs %lld entries, capacity %lld",
                    (long long)total, (long long)capacity);
    k_pl_scan<true><<<blocks_for(nb * 64), kBlock, 0, s>>>(g, x0, n, r2, reach, count, block_start,
                                                            slot);
    SPH_LAUNCHED();
    out->n = n;
    out->radius = radius;
    out->skin = grid->skin;
    out->count = count;
    out->block_start = block_start;
    out->slot = slot;
    out->capacity = capacity;
    out->x0 = x0;
    grid->pairs = out;
    return SPH_OK;
}
