// Internal helpers shared by the HIP sources of libsph (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "sph.h"

namespace sph {

// ------------------------------------------------------------------ errors --
int fail(int code, const char *fmt, ...);
void clear_error();

#define SPH_HIP_TRY(expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::sph::fail(SPH_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

#define SPH_LAUNCHED() SPH_HIP_TRY(hipGetLastError())

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n, int per_block = kBlock) {
    return (unsigned)((n + per_block - 1) / per_block);
}

// --------------------------------------------------------------- workspace --
// Every workspace starts with a 256-byte header whose first int32 is the device
// status flag; the rest is carved in 256-byte aligned pieces.  The same carving
// code computes sizes (base == nullptr) and pointers.
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Carve {
    char *base;
    size_t used = kAlign;  // header
    explicit Carve(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count) {
        T *r = base ? (T *)(base + used) : nullptr;
        used += align_up(count * sizeof(T));
        return r;
    }
    int32_t *status() const { return (int32_t *)base; }
};

__device__ inline void raise_flag(int32_t *status, int32_t code) { atomicCAS(status, 0, code); }

// Clears the status word (a kernel, not a memset, so the call sequence can be
// captured in a graph).
int clear_status(void *ws, hipStream_t s);

// --------------------------------------------------------------------- grid --
// Cell numbering.  Cells are grouped in tiles of 4 x 4 x 4 (x fastest inside a tile)
// and tiles in blocks of 4 x 4 x 4 tiles (16^3 cells, tiles in Morton order inside a
// block); blocks are numbered x fastest.  Slots follow the cell numbers, so 64
// consecutive slots (one wavefront of targets) fill a compact 3-D piece of a tile
// and the slots one XCD works on at a time a compact region, while runs of 4 cells
// along x stay contiguous for the row sweeps.
constexpr int kCellTile = 4;  // cells per tile edge
constexpr int kBlockC = 16;  // cells per block edge
constexpr int kBlockCells = kBlockC * kBlockC * kBlockC;

__host__ __device__ inline int32_t blocks_along(int32_t cells) { return (cells + kBlockC - 1) / kBlockC; }

// cell number of integer cell coordinates (nbx, nby: blocks along x and y)
__host__ __device__ inline int32_t cell_number(int ix, int iy, int iz, int nbx, int nby) {
    const int bx = ix >> 4, by = iy >> 4, bz = iz >> 4;
    const int tx = (ix >> 2) & 3, ty = (iy >> 2) & 3, tz = (iz >> 2) & 3;
    const int tile = (tx & 1) | ((ty & 1) << 1) | ((tz & 1) << 2) | ((tx >> 1) << 3) |
                     ((ty >> 1) << 4) | ((tz >> 1) << 5);
    const int local = (ix & 3) | ((iy & 3) << 2) | ((iz & 3) << 4);
    return ((bz * nby + by) * nbx + bx) * kBlockCells + tile * 64 + local;
}

// inverse of cell_number
__host__ __device__ inline void cell_coords(int32_t c, int nbx, int nby, int &ix, int &iy, int &iz) {
    const int b = c / kBlockCells, t = (c >> 6) & 63, l = c & 63;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tx = (t & 1) | (((t >> 3) & 1) << 1);
    const int ty = ((t >> 1) & 1) | (((t >> 4) & 1) << 1);
    const int tz = ((t >> 2) & 1) | (((t >> 5) & 1) << 1);
    ix = bx * kBlockC + tx * kCellTile + (l & 3);
    iy = by * kBlockC + ty * kCellTile + ((l >> 2) & 3);
    iz = bz * kBlockC + tz * kCellTile + (l >> 4);
}

struct GridDev {
    int32_t nx, ny, nz;
    int32_t nbx, nby;  // blocks of 16^3 cells along x and y
    double lox, loy, loz;
    double cell, inv_cell;
    double delta;  // tolerated movement since binning: skin / 2
    const int32_t *__restrict__ perm;
    // index of slot s in the state and output arrays: perm[s] (user order), or s
    // itself when the caller keeps its arrays in slot order (null)
    const int32_t *__restrict__ io;
    const int32_t *__restrict__ cell_start;
    const int32_t *__restrict__ cell_of;
    // frozen candidate-pair list (null count = none)
    const int32_t *__restrict__ pl_count;
    const int64_t *__restrict__ pl_block;
    const int32_t *__restrict__ pl_slot;
    const double *__restrict__ pl_x0;
    double pl_delta;  // tolerated movement since the list was built
};

inline GridDev grid_dev(const sph_grid *g) {
    GridDev d;
    d.nx = g->dims[0];
    d.ny = g->dims[1];
    d.nz = g->dims[2];
    d.nbx = blocks_along(d.nx);
    d.nby = blocks_along(d.ny);
    d.lox = g->lo[0];
    d.loy = g->lo[1];
    d.loz = g->lo[2];
    d.cell = g->cell;
    d.inv_cell = 1.0 / g->cell;
    d.delta = 0.5 * g->skin;
    d.perm = g->perm;
    d.io = g->perm;
    d.cell_start = g->cell_start;
    d.cell_of = g->cell_of;
    d.pl_count = g->pairs ? g->pairs->count : nullptr;
    d.pl_block = g->pairs ? g->pairs->block_start : nullptr;
    d.pl_slot = g->pairs ? g->pairs->slot : nullptr;
    d.pl_x0 = g->pairs ? g->pairs->x0 : nullptr;
    d.pl_delta = g->pairs ? 0.5 * g->pairs->skin : 0.0;
    return d;
}

int check_grid(const sph_grid *g);

__device__ inline int io_index(const GridDev &g, int64_t s) { return g.io ? g.io[s] : (int)s; }

__device__ inline int cell_index(double p, double lo, double inv_cell, int ncell) {
    double t = floor((p - lo) * inv_cell);
    t = fmin(fmax(t, 0.0), (double)(ncell - 1));  // NaN -> 0
    return (int)t;
}

// Distance from p to the slab of cell i along one axis; the first and last
// cells extend to infinity (they also hold the particles binned from outside
// the box).
__device__ inline double slab_gap(double p, double lo, double cell, int i, int ncell) {
    const double a = lo + cell * i;
    const double b = a + cell;
    double g = 0.0;
    if (i > 0 && p < a) g = a - p;
    if (i < ncell - 1 && p > b) g = p - b;
    return g;
}

// Squared distance of the partner test, every operation rounded on its own.
__device__ inline double dist2_exact(double xa, double ya, double za, double xb, double yb,
                                     double zb) {
#pragma clang fp contract(off)
    const double dx = xb - xa;
    const double dy = yb - ya;
    const double dz = zb - za;
    return (dx * dx + dy * dy) + dz * dz;
}

// Slot of logical workgroup for a 1-D launch of nblocks workgroups: the
// dispatcher deals workgroups to the 8 XCDs round robin; this remap gives each
// XCD one contiguous range of slots (neighbouring cells share its L2).
__device__ inline int64_t xcd_block(int64_t nblocks) {
    const int64_t i = blockIdx.x;
    const int64_t x = i & 7, q = nblocks >> 3, r = nblocks & 7;
    return x * q + (x < r ? x : r) + (i >> 3);
}

// Calls f(t) for every candidate slot t != s of slot s: from the pair list when
// the grid has one, otherwise by sweeping the cell rows within reach.
template <class F>
__device__ inline void for_each_candidate(const GridDev &g, int64_t s, double xa, double ya,
                                          double za, double reach, F &&f);

// Runs of consecutive cell numbers among the cells x0..x1 (x0 <= x1) of the row
// (iy, iz), in increasing x: f(c0, c1) for the cells numbered c0 .. c1 - 1 (a tile's
// run of 4 cells, and the next tile's when it follows in the numbering).
template <class F>
__device__ inline void for_each_cell_run(const GridDev &g, int iy, int iz, int x0, int x1, F &&f) {
    int x = x0;
    int cx = cell_number(x, iy, iz, g.nbx, g.nby);  // number of cell x
    int c0 = cx, c1 = cx;                            // the range being merged
    while (true) {
        const int e = min(x1, x | (kCellTile - 1));  // last cell of this tile's run
        c1 = cx + (e - x);
        x = e + 1;
        if (x > x1) break;
        cx = cell_number(x, iy, iz, g.nbx, g.nby);
        if (cx != c1 + 1) {
            f(c0, c1 + 1);
            c0 = cx;
        }
    }
    f(c0, c1 + 1);
}

// Slot ranges of the cells x0..x1 of the row (iy, iz), in increasing x, one per run
// of consecutive cell numbers.
template <class F>
__device__ inline void for_each_run(const GridDev &g, int iy, int iz, int x0, int x1, F &&f) {
    for_each_cell_run(g, iy, iz, x0, x1,
                      [&](int c0, int c1) { f(g.cell_start[c0], g.cell_start[c1]); });
}

// Visits the slot ranges [s0, s1) of every cell row whose box comes within
// `reach` of p (rows in y-z, the cells along x in runs of consecutive slots).
// A partner b of a target at p (|x_b - p| < h) lies within delta of its cell's
// box, so reach = (h + delta)(1 + 1e-9) visits every partner.  Rows go in
// increasing (z, y) and each row in increasing x, slots increasing inside a cell.
template <class F>
__device__ inline void for_each_row(const GridDev &g, double px, double py, double pz,
                                    double reach, F &&f) {
    const double r2 = reach * reach;
    const int z0 = cell_index(pz - reach, g.loz, g.inv_cell, g.nz);
    const int z1 = cell_index(pz + reach, g.loz, g.inv_cell, g.nz);
    const int y0 = cell_index(py - reach, g.loy, g.inv_cell, g.ny);
    const int y1 = cell_index(py + reach, g.loy, g.inv_cell, g.ny);
    for (int iz = z0; iz <= z1; ++iz) {
        const double gz = slab_gap(pz, g.loz, g.cell, iz, g.nz);
        const double gz2 = gz * gz;
        if (gz2 >= r2) continue;
        for (int iy = y0; iy <= y1; ++iy) {
            const double gy = slab_gap(py, g.loy, g.cell, iy, g.ny);
            const double d2 = gz2 + gy * gy;
            if (d2 >= r2) continue;
            const double w = sqrt(r2 - d2) * (1.0 + 1e-9);
            const int x0 = cell_index(px - w, g.lox, g.inv_cell, g.nx);
            const int x1 = cell_index(px + w, g.lox, g.inv_cell, g.nx);
            for_each_run(g, iy, iz, x0, x1, f);
        }
    }
}

// Staleness check of slot s at its current position: with a pair list, the
// particle must lie within the list's skin / 2 of its position when the list
// was built; otherwise within delta of the box of the cell it was binned into.
__device__ inline bool within_cell(const GridDev &g, int s, double x, double y, double z) {
    if (g.pl_count) {
        const double dx = x - g.pl_x0[3 * s], dy = y - g.pl_x0[3 * s + 1], dz = z - g.pl_x0[3 * s + 2];
        const double lim = g.pl_delta * (1.0 - 1e-9);
        return dx * dx + dy * dy + dz * dz <= lim * lim;
    }
    int ix, iy, iz;
    cell_coords(g.cell_of[s], g.nbx, g.nby, ix, iy, iz);
    const double lim = g.delta * (1.0 - 1e-9);
    return slab_gap(x, g.lox, g.cell, ix, g.nx) <= lim &&
           slab_gap(y, g.loy, g.cell, iy, g.ny) <= lim &&
           slab_gap(z, g.loz, g.cell, iz, g.nz) <= lim;
}

template <class F>
__device__ inline void for_each_candidate(const GridDev &g, int64_t s, double xa, double ya,
                                          double za, double reach, F &&f) {
    if (g.pl_count) {
        const int c = g.pl_count[s];
        const int32_t *p = g.pl_slot + g.pl_block[s >> 6] + (s & 63);
        for (int j = 0; j < c; ++j) f(p[(int64_t)j << 6]);
    } else {
        for_each_row(g, xa, ya, za, reach, [&](int s0, int s1) {
            for (int t = s0; t < s1; ++t)
                if (t != s) f(t);
        });
    }
}

// ------------------------------------------------------------ B-spline, 3-D --
// Section 3.1.1: W = s/h^3 w(q), dW/dr = 6s/h^4 g(q), q = r/h, s = 8/pi.
constexpr double kSigma3 = 2.5464790894703255;  // 8 / pi

// stable LSD radix sort of (uint64 key, int32 value) pairs by key bits [0, bits)
// (sort.hip); the result lands in buffer *which of the two
size_t radix_sort_tmp_elems(int64_t n);
int radix_sort_pairs(uint64_t *key[2], int32_t *val[2], int64_t n, int bits, int32_t *tmp,
                     int *which, hipStream_t s);

// exclusive scans (scan.hip)
int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s);
int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
size_t scan_tmp_elems(int64_t n);

}  // namespace sph
