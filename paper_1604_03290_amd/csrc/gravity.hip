// Barnes-Hut self-gravity with monopoles (section 3.3, eq. gravitational_force)
// on the octree of section 3.5.1.
//
// Instead of inserting particles under locks into a pointer octree, the tree is
// read off the Morton order of the particles: with 63-bit keys interleaving the
// 21-bit integer coordinates (x bit first in each triple), the cube of depth d
// holding a particle is its key's 3d-bit prefix, and the inner nodes (cubes with
// two or more particles) are the runs of equal prefixes of length >= 2 in the
// sorted keys.  Laid out in depth-first pre-order (children in octant order, the
// same order as the keys), the tree needs no child pointers: an item is followed
// by its first child, and each item stores `skip`, the first item after its
// subtree.  A node starting at sorted position i spans up to the first position
// whose key leaves its prefix (a binary search); the nodes starting at i are the
// depths D_{i-1} < d <= D_i, D_i being the depth shared by keys i and i + 1.
//
//   keys      bounding cube (reduction), integer coordinates, keys
//   sort      the library's stable LSD radix sort of (key, user index), 8 passes of
//             8 bits (sort.hip)
//   depth     D_i and the number of nodes starting at i; scan -> item offsets
//   items     leaves (position, mass) and inner nodes (depth, skip), and the list of
//             inner nodes (the k-th inner node in pre-order is list[k])
//   monopole  one pass per depth, deepest first, over the inner-node list: mass and
//             centre of mass of each node of that depth over its children in octant
//             order
//   walk      one wavefront walks the items for its 64 particles together: the
//             item pointer is uniform (its data arrive by scalar loads); a lane
//             that accepts a node resumes at the node's skip, and the wavefront
//             descends while any active lane needs to, so every lane takes exactly
//             the terms, and in the order, of its own walk.  Both possible next items
//             (t + 1 and the skip) are fetched while the current one is tested.
#include "common.hpp"
#include "rhs_common.hpp"
#include "timing.hpp"

namespace sph {
namespace {

// One 48-byte tree item (one base address for both scalar loads of the walk):
// pm = (x, y, z, m): a leaf's position and mass, an inner node's centre of mass and
// mass once the monopole pass ran; link = (skip, info), info = depth for an inner node
// and -1 - i for the leaf of sorted position i.
struct __attribute__((aligned(16))) Item {
    double4 pm;
    int2 link;
    int2 pad;
};

constexpr int kDepthMax = 21;  // 3 x 21 key bits

// ------------------------------------------------------------------ keys --
__global__ __launch_bounds__(kBlock) void k_bbox_partial(const double *__restrict__ x,
                                                         const double *__restrict__ y,
                                                         const double *__restrict__ z, int64_t n,
                                                         double *__restrict__ part) {
    __shared__ double lds[6][kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[6];
    if (i < n) {
        v[0] = v[3] = x[i];
        v[1] = v[4] = y[i];
        v[2] = v[5] = z[i];
    } else {
        const int64_t j = (int64_t)blockIdx.x * kBlock;  // first of the block, < n
        v[0] = v[3] = x[j];
        v[1] = v[4] = y[j];
        v[2] = v[5] = z[j];
    }
    for (int c = 0; c < 6; ++c) lds[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int c = 0; c < 3; ++c)
                lds[c][threadIdx.x] = fmin(lds[c][threadIdx.x], lds[c][threadIdx.x + w]);
            for (int c = 3; c < 6; ++c)
                lds[c][threadIdx.x] = fmax(lds[c][threadIdx.x], lds[c][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[(int64_t)blockIdx.x * 6 + threadIdx.x] = lds[threadIdx.x][0];
}

// box = (lo x, lo y, lo z, s0)
__global__ __launch_bounds__(kBlock) void k_bbox_final(const double *__restrict__ part,
                                                       int64_t nb, double *__restrict__ box) {
    __shared__ double lds[6][kBlock];
    double v[6];
    for (int c = 0; c < 6; ++c) v[c] = part[c];
    for (int64_t b = threadIdx.x; b < nb; b += kBlock)
        for (int c = 0; c < 6; ++c) {
            const double u = part[b * 6 + c];
            v[c] = c < 3 ? fmin(v[c], u) : fmax(v[c], u);
        }
    for (int c = 0; c < 6; ++c) lds[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int c = 0; c < 3; ++c)
                lds[c][threadIdx.x] = fmin(lds[c][threadIdx.x], lds[c][threadIdx.x + w]);
            for (int c = 3; c < 6; ++c)
                lds[c][threadIdx.x] = fmax(lds[c][threadIdx.x], lds[c][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double s0 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double e = lds[c + 3][0] - lds[c][0];
            if (e > s0) s0 = e;
        }
        box[0] = lds[0][0];
        box[1] = lds[1][0];
        box[2] = lds[2][0];
        box[3] = s0;
    }
}

__device__ inline uint32_t quantise(double v, double lo, double s0) {
    if (!(s0 > 0.0)) return 0u;
    const double u = floor((v - lo) / s0 * 2097152.0);  // 2^21
    if (!(u >= 0.0)) return 0u;  // a non-finite position (flagged by the caller)
    return u >= 2097152.0 ? 2097151u : (uint32_t)u;
}

// spreads the 21 low bits of v to every third bit
__device__ inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__global__ __launch_bounds__(kBlock) void k_keys(const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 const double *__restrict__ z,
                                                 const double *__restrict__ m, int64_t n,
                                                 const double *__restrict__ box,
                                                 uint64_t *__restrict__ key,
                                                 int32_t *__restrict__ idx,
                                                 int32_t *__restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i], mi = m[i];
    if (!isfinite(xi) || !isfinite(yi) || !isfinite(zi) || !(mi > 0.0) || !isfinite(mi))
        raise_flag(status, SPH_ERR_DOMAIN);
    const double s0 = box[3];
    const uint32_t qx = quantise(xi, box[0], s0), qy = quantise(yi, box[1], s0),
                   qz = quantise(zi, box[2], s0);
    key[i] = spread3(qx) << 2 | spread3(qy) << 1 | spread3(qz);
    idx[i] = (int32_t)i;
}

// ----------------------------------------------------------------- depth --
// depth shared by sorted keys i and i + 1 (-1 past the last); the number of inner
// nodes that start at i, c_i = max(0, D_i - D_{i-1}), and the deepest node's depth.
__device__ inline int shared_depth(const uint64_t *key, int64_t i, int64_t n) {
    if (i < 0) return -1;
    if (i + 1 >= n) return -1;
    const uint64_t d = key[i] ^ key[i + 1];
    const int bits = d ? __clzll((long long)d) - 1 : 63;  // common prefix of the 63-bit keys
    return bits / 3;
}

__global__ __launch_bounds__(kBlock) void k_depth(const uint64_t *__restrict__ key, int64_t n,
                                                  int64_t *__restrict__ cnt,
                                                  int32_t *__restrict__ max_depth) {
    __shared__ int bmax;
    if (threadIdx.x == 0) bmax = -1;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const int d1 = shared_depth(key, i, n), d0 = shared_depth(key, i - 1, n);
        cnt[i] = d1 > d0 ? d1 - d0 : 0;
        if (d1 >= 0) atomicMax(&bmax, d1);
    } else if (i == n) {
        cnt[n] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && bmax >= 0) atomicMax(max_depth, bmax);
}

// ----------------------------------------------------------------- items --
// Items of sorted position i: its inner nodes (depths D_{i-1} + 1 .. D_i), then its leaf.
__global__ __launch_bounds__(kBlock) void k_items(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ m, const uint64_t *__restrict__ key, const int32_t *__restrict__ idx,
    const int64_t *__restrict__ off, int64_t n, int32_t *__restrict__ list,
    Item *__restrict__ it) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int d1 = shared_depth(key, i, n), d0 = shared_depth(key, i - 1, n);
    const int64_t first = i + off[i];
    int64_t t = first;
    const uint64_t ki = key[i];
    for (int d = d0 + 1; d <= d1; ++d, ++t) {
        const int shift = 63 - 3 * d;
        const uint64_t pre = ki >> shift;
        int64_t lo = i + 1, hi = n;  // first position whose prefix differs
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if ((key[mid] >> shift) == pre)
                lo = mid + 1;
            else
                hi = mid;
        }
        it[t].link = make_int2((int)(lo + off[lo]), d);
        it[t].pm = make_double4(0.0, 0.0, 0.0, 0.0);
        list[off[i] + (t - first)] = (int32_t)t;
    }
    const int a = idx[i];
    it[t].link = make_int2((int)(t + 1), (int)(-1 - i));
    it[t].pm = make_double4(x[a], y[a], z[a], m[a]);
}

// -------------------------------------------------------------- monopole --
__global__ __launch_bounds__(kBlock) void k_monopole(const int32_t *__restrict__ list, int64_t K,
                                                     int depth, Item *__restrict__ it) {
#pragma clang fp contract(off)
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= K) return;
    const int t = list[j];
    const int2 lt = it[t].link;
    if (lt.y != depth) return;
    const int end = lt.x;
    double M = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (int c = t + 1; c < end; c = it[c].link.x) {
        const double4 p = it[c].pm;
        M = M + p.w;
        mx = mx + p.w * p.x;
        my = my + p.w * p.y;
        mz = mz + p.w * p.z;
    }
    it[t].pm = make_double4(mx / M, my / M, mz / M, M);
}

// ------------------------------------------------------------------ walk --
struct GravConsts {
    double G, th2, eps;  // th2 = theta^2
    int64_t n, T;
};

// a += G m_p (x_p - x_a) / (r + eps)^3 for r2 = r^2 > 0 (reciprocals by Newton steps
// from the hardware estimates)
__device__ inline void add_term(const GravConsts &k, double mp, double dx, double dy, double dz,
                                double r2, double &ax, double &ay, double &az) {
    if (r2 == 0.0) return;
    const double ir = rsqrt64(r2);
    double id;
    if (k.eps > 0.0) {
        id = rcp64(r2 * ir + k.eps);
    } else {
        id = ir;
    }
    const double f = k.G * mp * (id * id * id);
    ax = fma(f, dx, ax);
    ay = fma(f, dy, ay);
    az = fma(f, dz, az);
}

// The opening test s / r < theta is taken as s^2 < theta^2 r^2 with
// r^2 = (dx dx + dy dy) + dz dz rounded as written (no fused operations), the same
// arithmetic as the test's definition in the oracle.
__device__ inline double dist2_plain(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

__device__ inline bool opens_not(double s, double th2, double r2) {
#pragma clang fp contract(off)
    return s * s < th2 * r2;
}

__global__ __launch_bounds__(kBlock) void k_walk(GravConsts k, const double *__restrict__ box,
                                                 const int32_t *__restrict__ idx,
                                                 const Item *__restrict__ it,
                                                 const int64_t *__restrict__ off,
                                                 const int64_t *__restrict__ cnt,
                                                 double *__restrict__ ax_out,
                                                 double *__restrict__ ay_out,
                                                 double *__restrict__ az_out,
                                                 int32_t *__restrict__ count_out) {
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = i0 < k.n;
    const int64_t i = live ? i0 : k.n - 1;  // lanes past n walk the last particle, write nothing
    const double4 me = it[i + off[i] + cnt[i]].pm;
    const double xa = me.x, ya = me.y, za = me.z;
    const double s0 = box[3];
    double ax = 0.0, ay = 0.0, az = 0.0;
    int terms = 0;
    int resume = 0;
    const int T = (int)k.T;
    int t = 0;
    double4 p = it[0].pm;
    int2 l = it[0].link;
    while (t < T) {
        // both possible successors, fetched while this item is tested
        const int ta = min(t + 1, T - 1), tb = min(l.x, T - 1);
        const Item ia = it[ta], ib = it[tb];
        const double4 pa = ia.pm, pb = ib.pm;
        const int2 la = ia.link, lb = ib.link;
        const bool active = t >= resume;
        bool down = false;
        if (l.y >= 0) {
            const double dx = p.x - xa, dy = p.y - ya, dz = p.z - za;
            const double r2 = dist2_plain(dx, dy, dz);
            const bool take = active && opens_not(ldexp(s0, -l.y), k.th2, r2);
            if (take) {
                add_term(k, p.w, dx, dy, dz, r2, ax, ay, az);
                ++terms;
                resume = l.x;
            }
            down = __any(active && !take);
        } else if (active && -1 - l.y != i) {
            const double dx = p.x - xa, dy = p.y - ya, dz = p.z - za;
            add_term(k, p.w, dx, dy, dz, dist2_plain(dx, dy, dz), ax, ay, az);
            ++terms;
        }
        t = down ? t + 1 : l.x;
        p = down ? pa : pb;
        l = down ? la : lb;
    }
    if (!live) return;
    const int a = idx[i];
    ax_out[a] = ax;
    ay_out[a] = ay;
    az_out[a] = az;
    if (count_out) count_out[a] = terms;
}

__global__ void k_set_i32(int32_t *p, int32_t v) {
    if (threadIdx.x == 0) p[0] = v;
}

// ------------------------------------------------------------- workspace --
struct GravWs {
    double *part, *box;
    uint64_t *key[2];
    int32_t *idx[2];
    int64_t *cnt, *off, *scan_tmp;
    int32_t *max_depth;
    int32_t *list;
    Item *it;
    int32_t *sort_tmp;
};

int64_t node_capacity(int64_t n, int64_t cap) { return cap > 0 ? cap : 2 * n; }

GravWs carve_grav(Carve &c, int64_t n, int64_t cap) {
    GravWs w;
    w.part = c.take<double>((size_t)blocks_for(n) * 6);
    w.box = c.take<double>(4);
    for (int b = 0; b < 2; ++b) {
        w.key[b] = c.take<uint64_t>(n);
        w.idx[b] = c.take<int32_t>(n);
    }
    w.cnt = c.take<int64_t>(n + 1);
    w.off = c.take<int64_t>(n + 1);
    w.scan_tmp = c.take<int64_t>(scan_tmp_elems(n + 1));
    w.max_depth = c.take<int32_t>(1);
    w.list = c.take<int32_t>(cap);
    w.it = c.take<Item>(n + cap);
    w.sort_tmp = c.take<int32_t>(radix_sort_tmp_elems(n));
    return w;
}

}  // namespace

size_t gravity_ws_bytes(int64_t n, int64_t cap) {
    Carve c(nullptr);
    carve_grav(c, n, node_capacity(n, cap));
    return c.used;
}

}  // namespace sph

using namespace sph;

extern "C" int sph_gravity(const double *x, const double *y, const double *z, const double *m,
                           int64_t n, double G, double theta, double eps, double *ax, double *ay,
                           double *az, int32_t *count, int64_t node_cap, int64_t *nodes_out,
                           void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!x || !y || !z || !m || !ax || !ay || !az || !ws)
        return fail(SPH_ERR_INVALID_ARG, "null pointer");
    if (n < 1 || n > (int64_t)1 << 26) return fail(SPH_ERR_INVALID_ARG, "n must be in [1, 2^26]");
    if (!std::isfinite(G) || !std::isfinite(theta) || !std::isfinite(eps) || theta < 0.0 ||
        theta >= 1.0 || eps < 0.0)
        return fail(SPH_ERR_INVALID_ARG, "finite G, 0 <= theta < 1 and eps >= 0 required");
    const int64_t cap = node_capacity(n, node_cap);
    if (cap > 22 * n) return fail(SPH_ERR_INVALID_ARG, "node_cap above 22 n");
    const size_t need = gravity_ws_bytes(n, node_cap);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = clear_status(ws, s))) return rc;
    Carve c(ws);
    GravWs w = carve_grav(c, n, cap);
    TimedRegion tr("gravity", s);

    const unsigned nb = blocks_for(n);
    k_bbox_partial<<<nb, kBlock, 0, s>>>(x, y, z, n, w.part);
    SPH_LAUNCHED();
    k_bbox_final<<<1, kBlock, 0, s>>>(w.part, nb, w.box);
    SPH_LAUNCHED();
    k_keys<<<nb, kBlock, 0, s>>>(x, y, z, m, n, w.box, w.key[0], w.idx[0], c.status());
    SPH_LAUNCHED();

    int which = 0;
    if ((rc = radix_sort_pairs(w.key, w.idx, n, 63, w.sort_tmp, &which, s))) return rc;
    const uint64_t *key = w.key[which];
    const int32_t *idx = w.idx[which];

    k_set_i32<<<1, 64, 0, s>>>(w.max_depth, -1);
    SPH_LAUNCHED();
    k_depth<<<blocks_for(n + 1), kBlock, 0, s>>>(key, n, w.cnt, w.max_depth);
    SPH_LAUNCHED();
    if ((rc = exclusive_scan_i64(w.cnt, w.off, n + 1, w.scan_tmp, s))) return rc;

    // the tree's size: inner nodes K = off[n], and the deepest node's depth
    int64_t K = 0;
    int32_t dmax = -1;
    SPH_HIP_TRY(hipMemcpyAsync(&K, w.off + n, sizeof K, hipMemcpyDeviceToHost, s));
    SPH_HIP_TRY(hipMemcpyAsync(&dmax, w.max_depth, sizeof dmax, hipMemcpyDeviceToHost, s));
    SPH_HIP_TRY(hipStreamSynchronize(s));
    if (nodes_out) *nodes_out = K;
    if (K > cap)
        return fail(SPH_ERR_CAPACITY, "%lld inner nodes exceed capacity %lld", (long long)K,
                    (long long)cap);
    if (dmax > kDepthMax || (K > 0) != (dmax >= 0))
        return fail(SPH_ERR_HIP, "tree bookkeeping: depth %d with %lld nodes", dmax, (long long)K);

    k_items<<<nb, kBlock, 0, s>>>(x, y, z, m, key, idx, w.off, n, w.list, w.it);
    SPH_LAUNCHED();
    for (int d = dmax; d >= 0; --d) {
        k_monopole<<<blocks_for(K), kBlock, 0, s>>>(w.list, K, d, w.it);
        SPH_LAUNCHED();
    }
    const GravConsts k{G, theta * theta, eps, n, n + K};
    k_walk<<<nb, kBlock, 0, s>>>(k, w.box, idx, w.it, w.off, w.cnt, ax, ay, az, count);
    SPH_LAUNCHED();
    return SPH_OK;
}
