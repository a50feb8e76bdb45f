// Interaction partner lists (section 3.5.2) as a CSR in user order, each row
// ascending.  Positions are first gathered into slot order; a count pass takes
// candidates from the grid's pair list when it has one (else from the cell rows)
// and applies the exact test.  From the cell rows, one wavefront per row repeats the
// test over the row's candidates, packs the partners in LDS, sorts them in registers
// with a bitonic network and writes the row with whole-wavefront stores.  From the
// pair list, one wavefront per group of 64 slots writes the group's rows unsorted
// (tiles of the list in LDS, contiguous stores per row) and a second pass sorts each
// row in registers.  Rows longer than kRowMax are sorted afterwards in LDS.  When the
// list's build counted each slot's partners at this h and no position has changed
// since (bit for bit), those counts are the row lengths, and a slot whose candidates
// are all partners has its list written as its row without the test.
#include <climits>

#include "common.hpp"
#include "rhs_common.hpp"

namespace sph {
namespace {

constexpr int kSortMax = 1024;  // longest row sorted in LDS by one wavefront

// Gathers the positions into slot order; with a pair list also sets *moved when a
// position differs, bit for bit, from the list's build-time one.
__global__ __launch_bounds__(kBlock) void k_nb_gather(GridDev g, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, int64_t n,
                                                      double4 *__restrict__ pos,
                                                      int32_t *__restrict__ status,
                                                      int32_t *__restrict__ moved) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = g.perm[s];
    const double px = x[a], py = y[a], pz = z[a];
    if (!within_cell(g, (int)s, px, py, pz)) raise_flag(status, SPH_ERR_STALE_GRID);
    if (!(isfinite(px) && isfinite(py) && isfinite(pz))) raise_flag(status, SPH_ERR_DOMAIN);
    if (g.pl_x0) {
        const double *b = g.pl_x0 + 3 * s;
        if (__double_as_longlong(px) != __double_as_longlong(b[0]) ||
            __double_as_longlong(py) != __double_as_longlong(b[1]) ||
            __double_as_longlong(pz) != __double_as_longlong(b[2]))
            *moved = 1;
    }
    pos[s] = make_double4(px, py, pz, 0.0);
}

// partners of every slot (the exact test over its candidates), in user order.  known
// (the list's build-time partner counts, at this h) is taken instead when no position
// has moved since the list was built (*moved == 0): the same test on the same numbers.
__global__ __launch_bounds__(kBlock) void k_nb_count(GridDev g, const double4 *__restrict__ pos,
                                                     int64_t n, double h2, double reach,
                                                     int64_t *__restrict__ count,
                                                     const int32_t *__restrict__ known,
                                                     const int32_t *__restrict__ moved) {
    const int64_t s = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (s >= n) return;
    if (known && *moved == 0) {
        count[g.perm[s]] = known[s];
        return;
    }
    const double4 pa = pos[s];
    int64_t k = 0;
    for_each_candidate(g, s, pa.x, pa.y, pa.z, reach, [&](int t) {
        const double4 pb = pos[t];
        if (dist2_exact(pa.x, pa.y, pa.z, pb.x, pb.y, pb.z) < h2) ++k;
    });
    count[g.perm[s]] = k;
}

constexpr int kRowMax = 256;  // longest row sorted in registers (4 per lane)

// The value of lane (lane ^ J): lane-pair moves within a quad by DPP for J = 1, 2 (no
// LDS round trip), the swizzle unit's XOR mode inside 32 lanes for J = 4, 8, 16, and a
// backwards permute for J = 32.
template <int J>
__device__ inline int32_t xor_lane(int32_t v) {
    if constexpr (J == 1)
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    else if constexpr (J == 2)
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    else if constexpr (J == 4 || J == 8 || J == 16)
        return __builtin_amdgcn_ds_swizzle(v, 0x1F | (J << 10));  // and 31, or 0, xor J
    else
        return __shfl_xor(v, J);
}

// Bitonic sort, ascending, of the 64 E values v[e] held by one wavefront, value
// i = E lane + e (each lane holds E consecutive values): distances below E are
// exchanges inside a lane, the others between lanes (lane distance J / E).  bit[b] is
// bit b of the lane number, so a stage's directions are one or two of them.
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

template <int K, int E>
__device__ inline bool ascending(const bool (&bit)[6], int e) {
    // bit K of i = E lane + e: of e for K < E, else bit K / E of the lane (0 past 63)
    if constexpr (K < E) return (e & K) == 0;
    else if constexpr (K / E >= 64) return true;
    else return !bit[ilog2(K / E)];
}

template <int K, int J, int E>
__device__ inline void bitonic_stage(int32_t (&v)[E], const bool (&bit)[6]) {
    if constexpr (J < E) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int f = e ^ J;
            if (f > e) {
                const bool up = ascending<K, E>(bit, e);
                const int32_t a = v[e], b = v[f];
                const bool sw = (a > b) == up;  // (equal values may swap: alike)
                v[e] = sw ? b : a;
                v[f] = sw ? a : b;
            }
        }
    } else {
        constexpr int JL = J / E;
        // the lower index keeps the min when ascending, the max otherwise: the partner's
        // value where it is below (min) or not below (max) this one (equal values are
        // alike, so one compare and one select); lower: value i below its partner
        const bool take_max = !bit[ilog2(JL)] != ascending<K, E>(bit, 0);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int32_t o = xor_lane<JL>(v[e]);
            v[e] = ((o < v[e]) != take_max) ? o : v[e];
        }
    }
    if constexpr (J > 1) bitonic_stage<K, J / 2, E>(v, bit);
}

template <int K, int E>
__device__ inline void bitonic_merges(int32_t (&v)[E], const bool (&bit)[6]) {
    bitonic_stage<K, K / 2, E>(v, bit);
    if constexpr (K < 64 * E) bitonic_merges<2 * K, E>(v, bit);
}

template <int E>
__device__ inline void wave_bitonic(int32_t (&v)[E]) {
    const int lane = __lane_id();
    bool bit[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) bit[b] = (lane >> b) & 1;
    bitonic_merges<2, E>(v, bit);
}

template <int E>
__device__ inline void sort_store_row(const int32_t *buf, int len, int32_t *__restrict__ out) {
    const int lane = __lane_id();
    int32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * lane + e;
        v[e] = i < len ? buf[i] : INT_MAX;
    }
    wave_bitonic<E>(v);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * lane + e;
        if (i < len) out[i] = v[e];
    }
}

// Fill and sort, one wavefront per slot: the lanes test the slot's candidates 64 at
// a time and append the partners' user indices to an LDS buffer in candidate order
// (ballot prefix), then the row is sorted and stored.  Rows longer than kRowMax go
// to memory in candidate order for k_nb_sort.
__global__ __launch_bounds__(kBlock) void k_nb_rows(GridDev g, const double4 *__restrict__ pos,
                                                    int64_t n, double h2, double reach,
                                                    const int64_t *__restrict__ row_ptr,
                                                    int32_t *__restrict__ col) {
    __shared__ int32_t lds[kBlock / 64][kRowMax];
    int32_t *buf = lds[threadIdx.x >> 6];
    const int64_t s = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (s >= n) return;
    const int lane = __lane_id();
    const double4 pa = pos[s];
    const int a = g.perm[s];
    const int64_t r0 = row_ptr[a];
    const int len = (int)(row_ptr[a + 1] - r0);
    int32_t *out = col + r0;
    const bool big = len > kRowMax;
    int k = 0;  // partners found so far (wavefront-uniform)
    auto test = [&](int t, bool valid) {
        bool hit = false;
        int32_t u = 0;
        if (valid) {
            const double4 pb = pos[t];
            hit = dist2_exact(pa.x, pa.y, pa.z, pb.x, pb.y, pb.z) < h2;
            u = g.perm[t];
        }
        const unsigned long long m = __ballot(hit);
        if (hit) {
            const int at = k + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
            if (at < len) {  // the count pass found len partners with the same test
                if (big)
                    out[at] = u;
                else
                    buf[at] = u;
            }
        }
        k += __popcll(m);
    };
    if (g.pl_count) {
        const int c = g.pl_count[s];
        const int32_t *p = g.pl_slot + g.pl_block[s >> 6] + (s & 63);
        for (int j0 = 0; j0 < c; j0 += 64) {
            const int j = j0 + lane;
            test(j < c ? p[(int64_t)j << 6] : 0, j < c);
        }
    } else {
        for_each_row(g, pa.x, pa.y, pa.z, reach, [&](int s0, int s1) {
            for (int t0 = s0; t0 < s1; t0 += 64) {
                const int t = t0 + lane;
                test(t, t < s1 && t != (int)s);
            }
        });
    }
    if (big) return;
    wave_sync();
    if (len <= 64)
        sort_store_row<1>(buf, len, out);
    else if (len <= 128)
        sort_store_row<2>(buf, len, out);
    else
        sort_store_row<4>(buf, len, out);
}

// Fill over the frozen pair list, one wavefront per group of 64 slots.  The group's
// list is taken in tiles of 64 steps of 16 of its slots (64-byte pieces of the list's
// rows) into LDS; then for each slot of the tile in turn the lanes test 64 of its
// candidates (a column of the tile, conflict-free with the padded row length) and
// append the partners' user indices to its row in candidate order (ballot prefix, one
// contiguous store).  The rows are sorted afterwards by k_nb_sort_rows.  (A tile of all
// 64 slots would hold 16.6 KB of LDS per wavefront, two wavefronts per SIMD.)
constexpr int kTileSteps = 64;
constexpr int kTileRows = 16;
constexpr int kRowsInFlight = 8;  // rows whose user indices are gathered together
// a tile holds one step per lane: lane l tests step j0 + l of each row
static_assert(kTileSteps == 64, "the fill indexes a tile's steps by lane");

// lane r's value of a 64-bit quantity, as a scalar (r wavefront-uniform)
__device__ inline int64_t lane_value64(int64_t v, int r) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, r);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), r);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__global__ __launch_bounds__(kBlock) void k_nb_fill_list(GridDev g, const double4 *__restrict__ pos,
                                                         int64_t n, double h2,
                                                         const int64_t *__restrict__ row_ptr,
                                                         int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ known,
                                                         const int32_t *__restrict__ moved) {
    __shared__ int32_t lds[kBlock / 64][kTileSteps][kTileRows + 1];
    int32_t(*tile)[kTileRows + 1] = lds[threadIdx.x >> 6];
    const int lane = __lane_id();
    const int64_t nb = (n + 63) / 64;
    const int64_t B = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (B >= nb) return;
    const int64_t base = g.pl_block[B];
    const int64_t s = B * 64 + lane;
    const bool act = s < n;
    // this lane's row: candidates, output offset, length; k = partners written so far
    const int cnt = act ? g.pl_count[s] : 0;
    const int steps = list_steps(cnt);
    const int64_t r0 = act ? row_ptr[g.perm[s]] : 0;
    const int len = act ? (int)(row_ptr[g.perm[s] + 1] - r0) : 0;
    // every candidate of this slot is a partner (known at build time, positions
    // unchanged): its row is the list itself, written without the test
    const bool all = known && *moved == 0 && act && known[s] == cnt;
    int k = 0;
    const int rows = (int)min<int64_t>(64, n - B * 64);
    // every row of the group is its list: rows go kRowsInFlight at a time (as many gathers of user
    // indices in flight per lane)
    const bool group_all = __ballot(act && !all) == 0;
    for (int j0 = 0; j0 < steps; j0 += kTileSteps) {
        const int m = min(kTileSteps, steps - j0);
        for (int c0 = 0; c0 < rows; c0 += kTileRows) {
            const int c1 = min(rows, c0 + kTileRows);
            // tile[jj][i] = step j0 + jj of slot c0 + i (four steps per load)
            for (int e = lane; e < m * kTileRows; e += 64) {
                const int jj = e / kTileRows, i = e % kTileRows;
                tile[jj][i] = g.pl_slot[base + ((int64_t)(j0 + jj) << 6) + c0 + i];
            }
            wave_sync();
            if (group_all) {
                for (int r = c0; r < c1; r += kRowsInFlight) {
                    int cr[kRowsInFlight];
                    int32_t u[kRowsInFlight];
#pragma unroll
                    for (int q = 0; q < kRowsInFlight; ++q) {
                        cr[q] = r + q < rows ? __builtin_amdgcn_readlane(cnt, r + q) : 0;
                        u[q] = j0 + lane < cr[q] ? g.perm[tile[lane][r + q - c0]] : 0;
                    }
#pragma unroll
                    for (int q = 0; q < kRowsInFlight; ++q) {
                        if (j0 >= cr[q]) continue;  // wavefront-uniform (also past the rows)
                        const int64_t rr = lane_value64(r0, r + q);
                        const int kr = __builtin_amdgcn_readlane(k, r + q);
                        if (j0 + lane < cr[q]) col[rr + kr + lane] = u[q];
                    }
#pragma unroll
                    for (int q = 0; q < kRowsInFlight; ++q)
                        if (lane == r + q && j0 < cr[q]) k += min(64, cr[q] - j0);
                }
                wave_sync();
                continue;
            }
            for (int r = c0; r < c1; ++r) {  // row r's values come from lane r (scalar reads)
                const int cr = __builtin_amdgcn_readlane(cnt, r);
                if (j0 >= cr) continue;  // wavefront-uniform
                const int64_t sr = B * 64 + r;
                const bool valid = j0 + lane < cr;
                const int kr = __builtin_amdgcn_readlane(k, r);
                const int64_t rr = lane_value64(r0, r);
                if (__builtin_amdgcn_readlane((int)all, r)) {
                    // lanes 0 .. min(64, cr - j0) - 1 all hit
                    if (valid) col[rr + kr + lane] = g.perm[tile[lane][r - c0]];
                    if (lane == r) k += min(64, cr - j0);
                    continue;
                }
                const double4 pa = pos[sr];
                bool hit = false;
                int32_t u = 0;
                if (valid) {
                    const int t = tile[lane][r - c0];
                    const double4 pb = pos[t];
                    hit = dist2_exact(pa.x, pa.y, pa.z, pb.x, pb.y, pb.z) < h2;
                    u = g.perm[t];
                }
                const unsigned long long mk = __ballot(hit);
                const int lr = __builtin_amdgcn_readlane(len, r);
                if (hit) {
                    const int at = kr + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0));
                    if (at < lr) col[rr + at] = u;  // the count pass found lr with the same test
                }
                if (lane == r) k += __popcll(mk);
            }
            wave_sync();
        }
    }
}

// One wavefront per row: the row (in candidate order) sorted ascending in registers
// with the bitonic network (rows up to kRowMax; 1, 2 or 4 values per lane) and
// written back; a row already in order is left as it is.  Longer rows are left to
// k_nb_sort.
template <int E>
__device__ inline void sort_row_inplace(int32_t *__restrict__ row, int len) {
    const int lane = __lane_id();
    int32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * lane + e;
        v[e] = i < len ? row[i] : INT_MAX;
    }
    // in order already? (value i <= value i + 1 for every i)
    bool ok = true;
#pragma unroll
    for (int e = 0; e + 1 < E; ++e) ok = ok && v[e] <= v[e + 1];
    const int32_t nxt = __shfl_down(v[0], 1);  // the next lane's first
    ok = ok && (lane == 63 || v[E - 1] <= nxt);
    if (__ballot(!ok) == 0) return;
    wave_bitonic<E>(v);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * lane + e;
        if (i < len) row[i] = v[e];
    }
}

// Bitonic sort of one row in LDS by one wavefront (buf: kSortMax values); rows longer
// than kSortMax, which no workload here produces, fall back to an insertion sort by
// lane 0.
__device__ inline void sort_long_row(int32_t *__restrict__ row, int len, int32_t *buf) {
    const int lane = __lane_id();
    if (len > kSortMax) {
        if (lane == 0) {
            for (int64_t i = 1; i < len; ++i) {
                const int32_t v = row[i];
                int64_t j = i - 1;
                while (j >= 0 && row[j] > v) {
                    row[j + 1] = row[j];
                    --j;
                }
                row[j + 1] = v;
            }
        }
        return;
    }
    int n2 = 2;
    while (n2 < len) n2 <<= 1;
    for (int i = lane; i < n2; i += 64) buf[i] = i < len ? row[i] : INT_MAX;
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
    for (int i = lane; i < len; i += 64) row[i] = buf[i];
}

// Every row of the CSR, one wavefront per row: in registers up to kRowMax values, in
// LDS beyond.
__global__ __launch_bounds__(kBlock) void k_nb_sort_rows(const int64_t *__restrict__ row_ptr,
                                                         int64_t n, int32_t *__restrict__ col) {
    __shared__ int32_t lds[kBlock / 64][kSortMax];
    const int64_t a = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (a >= n) return;
    const int64_t r0 = row_ptr[a];
    const int len = (int)(row_ptr[a + 1] - r0);
    if (len <= 1) return;
    if (len <= 64)
        sort_row_inplace<1>(col + r0, len);
    else if (len <= 128)
        sort_row_inplace<2>(col + r0, len);
    else if (len <= kRowMax)
        sort_row_inplace<4>(col + r0, len);
    else
        sort_long_row(col + r0, len, lds[threadIdx.x >> 6]);
}

// the rows longer than min_len (which k_nb_rows leaves unsorted), one wavefront per row
__global__ __launch_bounds__(kBlock) void k_nb_sort(const int64_t *__restrict__ row_ptr,
                                                    int64_t n, int32_t *__restrict__ col,
                                                    int min_len) {
    __shared__ int32_t lds[kBlock / 64][kSortMax];
    const int64_t a = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (a >= n) return;
    const int64_t r0 = row_ptr[a];
    const int len = (int)(row_ptr[a + 1] - r0);
    if (len <= 1 || len <= min_len) return;  // shorter rows are sorted already
    sort_long_row(col + r0, len, lds[threadIdx.x >> 6]);
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
    // with a pair list whose build counted partners at this h: its counts, and its lists
    // as rows, where no position has changed since
    const int32_t *known =
        g.pl_count && grid->pairs->partners && h == grid->h ? grid->pairs->partners : nullptr;
    int32_t *moved = c.status() + 1;  // the header's second word, cleared with the flag
    k_nb_gather<<<blocks_for(n), kBlock, 0, s>>>(g, x, y, z, n, pos, c.status(), moved);
    SPH_LAUNCHED();
    k_nb_count<<<blocks_for(n), kBlock, 0, s>>>(g, pos, n, h * h, reach, count, known, moved);
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
    if (nnz == 0) return SPH_OK;
    if (g.pl_count) {
        k_nb_fill_list<<<blocks_for((n + 63) / 64, kBlock / 64), kBlock, 0, s>>>(g, pos, n, h * h,
                                                                                row_ptr, col, known,
                                                                                moved);
        SPH_LAUNCHED();
        k_nb_sort_rows<<<blocks_for(n, kBlock / 64), kBlock, 0, s>>>(row_ptr, n, col);
        SPH_LAUNCHED();
    } else {
        k_nb_rows<<<blocks_for(n, kBlock / 64), kBlock, 0, s>>>(g, pos, n, h * h, reach, row_ptr, col);
        SPH_LAUNCHED();
        k_nb_sort<<<blocks_for(n, kBlock / 64), kBlock, 0, s>>>(row_ptr, n, col, kRowMax);
        SPH_LAUNCHED();
    }
    return SPH_OK;
}
