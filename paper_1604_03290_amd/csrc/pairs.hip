// Frozen candidate-pair list ("interactionsList" of section 3.5.2 with a
// skin): for every slot, the slots whose distance was below h + skin when the
// list was built.  While every particle stays within skin/2 of its position at
// build time this is a superset of its partners, and the pair kernels re-test
// d^2 < h^2 exactly at the current positions.
//
// Layout: slots are grouped in blocks of 64 (one wavefront); inside block B the
// j-th candidate of the block's lane l sits at slot[block_start[B] + 64 j + l],
// so the j-th loads of a wavefront are contiguous.  Each block's lists are padded to
// its longest, whose length (the largest count of its 64 slots) is the block's number
// of steps.  A block's room, 64 times the largest bound of its slots (the slots of the
// cells within reach of each slot, counted without a distance test), is fixed before
// the one pass that tests and writes the candidates, so no count pass is needed.
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

// Distance from the interval [b0, b1] to the slab of cell i along one axis (the
// first and last cells extend to infinity, as in slab_gap).
__device__ inline double box_gap(double b0, double b1, double lo, double cell, int i, int ncell) {
    const double a = lo + cell * i;
    const double b = a + cell;
    double g = 0.0;
    if (i > 0 && b1 < a) g = a - b1;
    if (i < ncell - 1 && b0 > b) g = b0 - b;
    return g;
}

__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Upper bound of every slot's candidates: the slots of the cells within reach of its
// position (each candidate lies in one of them, within delta of its cell's box), self
// included.
__global__ __launch_bounds__(kBlock) void k_pl_bound(GridDev g, const double *__restrict__ x0,
                                                     int64_t n, double reach,
                                                     int32_t *__restrict__ bound) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int b = 0;
    for_each_row(g, x0[3 * s], x0[3 * s + 1], x0[3 * s + 2], reach,
                 [&](int s0, int s1) { b += s1 - s0; });
    bound[s] = b;
}

// Fill pass, one wavefront per group of 64 slots.  The fill writes entry j of lane l
// at block_start[B] + 64 j + l, pads every list to the group's longest with the slot
// itself (n - 1 for the lanes past n), so every entry of a group's steps is a valid
// slot and readers of whole groups load without guards, and writes each slot's count
// (and its partners at the grid's h).
//
// A compact group sweeps, once and cooperatively, the cell rows of its bounding box
// widened by the reach, from the middle of the region outwards (z, then y), x
// increasing along a row and slots increasing inside a cell; each list holds its
// slot's candidates in that order.  The sweep goes in passes of up to 64 rows: each
// lane takes one row (culled against the group's box as a whole) and lays the row's
// runs of consecutive slots out in LDS, in row order; the pass's candidates are then
// streamed 64 at a time, so that the loads of a pass do not wait on one another row by
// row.  Each loaded candidate is culled, one lane per candidate, against the group's
// box widened by the radius (one farther away is no lane's candidate); the survivors
// are packed in order into an LDS buffer, which the 64 lanes test against their own
// slots 64 candidates at a time (broadcast reads).  A group spread over a region of
// more than kSpread times one slot's cells (sparse parts of a set) sweeps per lane
// instead, in the order of for_each_row.
constexpr double kSpread = 8.0;
constexpr int kRunCap = 256;  // runs of one pass (LDS)

__global__ __launch_bounds__(kBlock) void k_pl_fill(GridDev g, const double *__restrict__ x0,
                                                    int64_t n, double r2, double reach,
                                                    int32_t *__restrict__ count,
                                                    const int64_t *__restrict__ block_start,
                                                    int32_t *__restrict__ slot, double h2,
                                                    int32_t *__restrict__ partners) {
    __shared__ double lds[kBlock / 64][3][2 * kWave];
    __shared__ int32_t lds_t[kBlock / 64][2 * kWave];
    __shared__ int32_t lds_r[kBlock / 64][2][kRunCap];
    double(*cand)[2 * kWave] = lds[threadIdx.x >> 6];
    int32_t *cand_t = lds_t[threadIdx.x >> 6];
    int32_t *run_s0 = lds_r[threadIdx.x >> 6][0];   // a run's first slot (first its cell)
    int32_t *run_pre = lds_r[threadIdx.x >> 6][1];  // candidates before it in the pass
    const int lane = __lane_id();
    const int64_t nb = (n + kWave - 1) / kWave;
    const int64_t B = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    if (B >= nb) return;  // whole wavefront past the end
    const int64_t s = B * kWave + lane;
    const bool act = s < n;
    const int64_t sa = act ? s : B * kWave;  // lanes past n stand on the group's first slot
    const double xa = x0[3 * sa], ya = x0[3 * sa + 1], za = x0[3 * sa + 2];
    const int64_t base = block_start[B] + lane;
    const int64_t room = (block_start[B + 1] - block_start[B]) / kWave;
    int c = 0, np = 0;  // candidates and partners (d^2 < h^2) among them
    int32_t *const group = slot + block_start[B];  // entry j of lane l at group[64 j + l]
    const int iroom = (int)min(room, (int64_t)(INT_MAX >> 6));
    auto hit = [&](int t, double d) {
        // the bound pass gave room for every candidate; the guard keeps a write
        // inside the group even so
        if (c < iroom) group[(uint32_t)((c << 6) + lane)] = t;
        np += d < h2;
        ++c;
    };
    const double bx0 = wave_min(xa), bx1 = wave_max(xa);
    const double by0 = wave_min(ya), by1 = wave_max(ya);
    const double bz0 = wave_min(za), bz1 = wave_max(za);
    const int z0 = cell_index(bz0 - reach, g.loz, g.inv_cell, g.nz);
    const int z1 = cell_index(bz1 + reach, g.loz, g.inv_cell, g.nz);
    const int y0 = cell_index(by0 - reach, g.loy, g.inv_cell, g.ny);
    const int y1 = cell_index(by1 + reach, g.loy, g.inv_cell, g.ny);
    const int x0c = cell_index(bx0 - reach, g.lox, g.inv_cell, g.nx);
    const int x1c = cell_index(bx1 + reach, g.lox, g.inv_cell, g.nx);
    const double own = 2.0 * reach * g.inv_cell + 1.0;  // cells along one axis of one slot
    const double box = (double)(x1c - x0c + 1) * (y1 - y0 + 1) * (z1 - z0 + 1);
    if (box > kSpread * own * own * own) {
        if (act)
            for_each_row(g, xa, ya, za, reach, [&](int s0, int s1) {
                for (int t = s0; t < s1; ++t) {
                    if (t == s) continue;
                    const double d = dist2_exact(xa, ya, za, x0[3 * t], x0[3 * t + 1], x0[3 * t + 2]);
                    if (d < r2) hit(t, d);
                }
            });
    } else {
        const double rr = reach * reach;
        // the cull keeps every candidate within the radius of a point of the box, with a
        // margin far above the rounding of either distance
        const double rb2 = r2 * (1.0 + 1e-6);
        int pend = 0;  // candidates waiting in the buffer (wavefront-uniform)
        auto test = [&](int m) {
            int k = 0;
            for (; k + 4 <= m; k += 4) {  // four distances, then their hits
                int t[4];
                double d[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    t[q] = cand_t[k + q];
                    d[q] = dist2_exact(xa, ya, za, cand[0][k + q], cand[1][k + q], cand[2][k + q]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (act && d[q] < r2 && t[q] != (int)s) hit(t[q], d[q]);
            }
            for (; k < m; ++k) {
                const int t = cand_t[k];
                const double d = dist2_exact(xa, ya, za, cand[0][k], cand[1][k], cand[2][k]);
                if (act && d < r2 && t != (int)s) hit(t, d);
            }
        };
        // one candidate per lane (t, where valid): loaded, culled, packed behind the
        // waiting ones; 64 waiting are tested
        auto push = [&](bool valid, int t) {
            bool keep = false;
            double px = 0.0, py = 0.0, pz = 0.0;
            if (valid) {
                px = x0[3 * (int64_t)t];
                py = x0[3 * (int64_t)t + 1];
                pz = x0[3 * (int64_t)t + 2];
                const double ex = fmax(fmax(bx0 - px, px - bx1), 0.0);
                const double ey = fmax(fmax(by0 - py, py - by1), 0.0);
                const double ez = fmax(fmax(bz0 - pz, pz - bz1), 0.0);
                keep = ex * ex + ey * ey + ez * ez < rb2;
            }
            const unsigned long long mk = __ballot(keep);
            if (keep) {
                const int at = pend + (int)__builtin_amdgcn_mbcnt_hi(
                                          (unsigned)(mk >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0));
                cand[0][at] = px;
                cand[1][at] = py;
                cand[2][at] = pz;
                cand_t[at] = t;
            }
            pend += __popcll(mk);
            wave_sync();
            if (pend >= kWave) {
                test(kWave);
                pend -= kWave;
                wave_sync();
                if (lane < pend) {  // the rest to the front (reads above kWave only)
                    cand[0][lane] = cand[0][kWave + lane];
                    cand[1][lane] = cand[1][kWave + lane];
                    cand[2][lane] = cand[2][kWave + lane];
                    cand_t[lane] = cand_t[kWave + lane];
                }
                wave_sync();
            }
        };
        // rows from the middle of the region outwards (z, then y): the lanes of the
        // group then meet their partners at more even rates, so that the rows of the
        // list they fill together are completed sooner.  Row rank r: z the r / ny-th
        // and y the r % ny-th of that order.
        const int nzr = z1 - z0 + 1, nyr = y1 - y0 + 1, nrows = nzr * nyr;
        auto middle_out = [](int r, int lo, int hi) {  // r-th of c, c - 1, c + 1, c - 2, ...
            const int c = (lo + hi) >> 1, a = c - lo;
            return r <= 2 * a ? c + ((r & 1) ? -((r + 1) >> 1) : (r >> 1)) : hi;
        };
        for (int rb = 0; rb < nrows;) {
            // this lane's row of the pass: its cells in x and its number of runs
            const int r = rb + lane;
            int iy = 0, iz = 0, xr0 = 0, xr1 = -1, nr = 0;
            if (r < nrows) {
                iz = middle_out(r / nyr, z0, z1);
                iy = middle_out(r % nyr, y0, y1);
                const double gz = box_gap(bz0, bz1, g.loz, g.cell, iz, g.nz);
                const double gy = box_gap(by0, by1, g.loy, g.cell, iy, g.ny);
                const double d2 = gz * gz + gy * gy;
                if (gz * gz < rr && d2 < rr) {
                    const double w = sqrt(rr - d2) * (1.0 + 1e-9);
                    xr0 = cell_index(bx0 - w, g.lox, g.inv_cell, g.nx);
                    xr1 = cell_index(bx1 + w, g.lox, g.inv_cell, g.nx);
                    for_each_cell_run(g, iy, iz, xr0, xr1, [&](int, int) { ++nr; });
                }
            }
            // runs before this lane's (exclusive scan over the lanes)
            int off = nr;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(off, o);
                if (lane >= o) off += v;
            }
            off -= nr;
            // the rows that fit the pass: a prefix of the lanes
            const int take = __popcll(__ballot(r < nrows && off + nr <= kRunCap));
            if (take == 0) {
                // a single row with more runs than a pass holds: its runs one by one
                const int fy = __builtin_amdgcn_readfirstlane(iy), fz = __builtin_amdgcn_readfirstlane(iz);
                const int f0 = __builtin_amdgcn_readfirstlane(xr0), f1 = __builtin_amdgcn_readfirstlane(xr1);
                for_each_run(g, fy, fz, f0, f1, [&](int s0, int s1) {
                    for (int t0 = s0; t0 < s1; t0 += kWave) push(t0 + lane < s1, t0 + lane);
                });
                rb += 1;
                continue;
            }
            const int nrun = __shfl(off + nr, take - 1);
            if (lane < take && nr > 0) {  // (a culled row has no runs)
                int j = off;
                for_each_cell_run(g, iy, iz, xr0, xr1, [&](int c0, int c1) {
                    run_s0[j] = c0;
                    run_pre[j] = c1;
                    ++j;
                });
            }
            wave_sync();
            // the runs' slots: cells to slot ranges, and their lengths scanned
            int len[kRunCap / kWave], sum = 0;
#pragma unroll
            for (int q = 0; q < kRunCap / kWave; ++q) {
                const int j = kRunCap / kWave * lane + q;
                len[q] = 0;
                if (j < nrun) {
                    const int s0 = g.cell_start[run_s0[j]];
                    len[q] = g.cell_start[run_pre[j]] - s0;
                    run_s0[j] = s0;
                }
                sum += len[q];
            }
            int before = sum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(before, o);
                if (lane >= o) before += v;
            }
            const int total = __shfl(before, 63);
            before -= sum;
#pragma unroll
            for (int q = 0; q < kRunCap / kWave; ++q) {
                const int j = kRunCap / kWave * lane + q;
                if (j < nrun) run_pre[j] = before;
                before += len[q];
            }
            wave_sync();
            // the pass's candidates in order, 64 at a time (run of candidate f: the last
            // with run_pre <= f)
            for (int f0 = 0; f0 < total; f0 += kWave) {
                const int f = f0 + lane;
                int lo = 0, hi = nrun;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (run_pre[mid] <= f) lo = mid; else hi = mid;
                }
                push(f < total, run_s0[lo] + (f - run_pre[lo]));
            }
            wave_sync();
            rb += take;
        }
        test(pend);
    }
    // the group's steps: its longest list (at most its room)
    int steps = min((int64_t)c, room);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) steps = max(steps, __shfl_xor(steps, o));
    const int32_t pad = act ? (int32_t)s : (int32_t)(n - 1);
    for (int64_t j = c; j < steps; ++j) slot[base + kWave * j] = pad;
    if (act) {
        count[s] = c;
        if (partners) partners[s] = np;
    }
}

// sizes[B] = 64 * (largest bound of block B)
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
                               sph_pairs *out, int32_t *count, int32_t *partners,
                               int64_t *block_start, int32_t *slot, int64_t capacity, double *x0,
                               int64_t *needed, void *ws, size_t ws_bytes, void *stream) {
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
    const double h2 = grid->h * grid->h;  // the partner test of sph_neighbours at grid->h
    // bounds into count (the fill overwrites them with the counts)
    k_pl_bound<<<blocks_for(n), kBlock, 0, s>>>(g, x0, n, reach, count);
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
    k_pl_fill<<<blocks_for(nb, kBlock / 64), kBlock, 0, s>>>(g, x0, n, r2, reach, count,
                                                              block_start, slot, h2, partners);
    SPH_LAUNCHED();
    out->n = n;
    out->radius = radius;
    out->skin = grid->skin;
    out->count = count;
    out->block_start = block_start;
    out->slot = slot;
    out->capacity = capacity;
    out->x0 = x0;
    out->partners = partners;
    grid->pairs = out;
    return SPH_OK;
}
