// Right-hand side of the SPH solid-body equations.
//
//   prepass   per slot, FP64: gather the particle's state into slot order,
//             pressure (section 2.5.1), von Mises factor (section 2.6),
//             T = sigma / rho^2 with sigma = -p I + f_Y S (section 2.2),
//             V = m / rho; stale-grid and domain checks
//   pairs     per target slot: partner test d^2 < h^2 (section 3.5.2) over the
//             cell rows within reach; density sum (eq. density_by_kernel_sum),
//             velocity gradient L (section 3.1.6), acceleration with the
//             artificial viscosity Pi* (eqs. accel, accel_artvisc, section 3.1.3)
//   postpass  fused into the pair kernel's epilogue, FP64: drho = -rho tr L
//             (eq. continuity_equation_sph), Hooke + Jaumann stress rate
//             (section 2.4), scatter to user order
//
// Cubic B-spline (section 3.1.1) with q = r/h:  W = s/h^3 w(q) and
// W'(r)/r = 6 s/h^5 f(q) with w = 1 - 6q^2 + 6q^3, f = 3q - 2 for q < 1/2 and
// w = 2 (1-q)^3, f = -(1-q)^2 / q for 1/2 <= q < 1, so grad_a W_ab =
// (W'/r)(x_a - x_b) stays finite as r -> 0.
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "rhs_common.hpp"
#include "timing.hpp"

namespace sph {
namespace {

// --------------------------------------------------------------- prepass --
// the slot of every user index: inv[perm[s]] = s
__global__ __launch_bounds__(kBlock) void k_invert(const int32_t *__restrict__ perm, int64_t n,
                                                   int32_t *__restrict__ inv) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) inv[perm[s]] = (int32_t)s;
}

// dd3 / nact (null unless requested): the damage model's rates (section 3.2).  With
// inv (user-order state, its inverse permutation) thread i takes user particle i, so
// the state arrays are read in order and each thread writes its slot's whole 128-byte
// record; without it (slot-ordered state) thread i takes slot i.
__global__ __launch_bounds__(kBlock) void k_prepass(GridDev g, StateDev st, int64_t n, Consts k,
                                                    double *__restrict__ rec,
                                                    int32_t *__restrict__ status, double *dd3,
                                                    int32_t *nact, const int32_t *__restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = inv ? (int64_t)inv[i] : i;
    const int a = inv ? (int)i : io_index(g, s);
    const double S[6] = {st.sxx[a], st.syy[a], st.szz[a], st.sxy[a], st.sxz[a], st.syz[a]};
    const double d = st.d ? st.d[a] : 0.0, rho = st.rho[a], m = st.m[a];
    const double p = write_rec(g, k, s, st.x[a], st.y[a], st.z[a], st.vx[a], st.vy[a], st.vz[a],
                               rho, S, m, rec, status, st.u ? st.u[a] : 0.0, d);
    if (dd3) {
        const double f = (1.0 - d) * yield_factor(k, S);
        const double ph = p >= 0.0 ? p : (1.0 - d) * p;
        const double sig[6] = {f * S[0] - ph, f * S[1] - ph, f * S[2] - ph,
                               f * S[3],      f * S[4],      f * S[5]};
        damage_rate(k, st, n, a, sig, rho, m, d, dd3, nact, status);
    }
}

// FP32 copies of the pair operands (positions stay FP64 for the exact test), 80 bytes:
//   x y | z (vx vy) | (vz rho m V) | (T0 T1 T2 T3) | (T4 T5 c -)
// c being the record's signed sound speed.
__global__ __launch_bounds__(kBlock) void k_narrow(const double *__restrict__ rec, int64_t n,
                                                   float *__restrict__ r32) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double *r = rec + s * kRec;
    char *o = reinterpret_cast<char *>(r32) + s * kRec32Bytes;
    *reinterpret_cast<double2 *>(o) = make_double2(r[0], r[1]);
    *reinterpret_cast<double *>(o + 16) = r[2];
    *reinterpret_cast<float2 *>(o + 24) = make_float2((float)r[3], (float)r[4]);
    *reinterpret_cast<float4 *>(o + 32) = make_float4((float)r[5], (float)r[6], (float)r[14], (float)r[7]);
    *reinterpret_cast<float4 *>(o + 48) = make_float4((float)r[8], (float)r[9], (float)r[10], (float)r[11]);
    *reinterpret_cast<float4 *>(o + 64) = make_float4((float)r[12], (float)r[13], (float)r[15], 0.0f);
}

// ---------------------------------------------------------- pairs, FP64 --
template <bool kCorr, bool kExt>
__global__ __launch_bounds__(kBlock) void k_pairs64(GridDev g, int64_t n, Consts k,
                                                    const double *__restrict__ rec, StateDev st,
                                                    OutDev out, double *__restrict__ Lout) {
    const int64_t s = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (s >= n) return;
    const double2 *ra = rec2(rec, s);
    const double2 p0 = ra[0], p1 = ra[1], p2 = ra[2], p3 = ra[3], p4 = ra[4], p5 = ra[5], p6 = ra[6];
    const double xa = p0.x, ya = p0.y, za = p1.x, vxa = p1.y, vya = p2.x, vza = p2.y;
    const double rho_a = p3.x;
    Acc64 acc;
    acc.rs = ra[7].x * k.Wn;  // own term m_a W(0)
    const double c_a = ra[7].y;
    const double Ta[6] = {p4.x, p4.y, p5.x, p5.y, p6.x, p6.y};
    const bool tens_a = kExt && signbit(c_a);
    for_each_candidate(g, s, xa, ya, za, k.reach, [&](int t) {
        const double2 *rb = rec2(rec, t);
        const double2 b0 = rb[0], b1 = rb[1];
        const double d2 = dist2_exact(xa, ya, za, b0.x, b0.y, b1.x);
        if (!(d2 < k.h2)) return;
        const double2 b2 = rb[2], b3 = rb[3], b4 = rb[4], b5 = rb[5], b6 = rb[6], b7 = rb[7];
        const double Tb[6] = {b4.x, b4.y, b5.x, b5.y, b6.x, b6.y};
        pair64<kCorr, kExt>(k, d2, xa - b0.x, ya - b0.y, za - b1.x, b1.y - vxa, b2.x - vya,
                            b2.y - vza, rho_a, b3.x, p4.x + b4.x, p4.y + b4.y, p5.x + b5.x,
                            p5.y + b5.y, p6.x + b6.x, p6.y + b6.y, b7.x, b3.y, acc, Ta, Tb, tens_a,
                            c_a, b7.y);
    });
    postpass(k, io_index(g, s), rho_a, acc.L, acc.ax, acc.ay, acc.az, acc.rs, st, out,
             kCorr ? acc.M : nullptr);
    if (kExt) postpass_ext(k, io_index(g, s), acc, st, out);
    if (Lout) store_vgrad<kCorr>(Lout, s, acc.L, acc.M);
}

// FP64 pair sums over the frozen pair list: a workgroup of kSplit wavefronts takes one
// block of 64 slots, wavefront q walking the 64 lists in lock step over steps q,
// q + kSplit, ... and gathering the 64 partner records of each step cooperatively;
// the partial sums are folded into wavefront 0, which runs the postpass.
template <bool kCorr, bool kExt>
__global__ __launch_bounds__(64 * kSplit) void k_pairs64_list(GridDev g, int64_t n, Consts k,
                                                              const double *__restrict__ rec,
                                                              StateDev st, OutDev out,
                                                              double *__restrict__ Lout) {
    __shared__ double2 lbuf[kSplit][64 * 8];
    const int q = threadIdx.x >> 6;
    double2 *buf = lbuf[q];
    const int64_t w = xcd_block(gridDim.x);
    const int64_t w0 = w * 64;
    if (w0 >= n) return;  // whole workgroup past the end
    const int64_t s = w0 + __lane_id();
    const bool act = s < n;
    const int64_t base = g.pl_block[w];
    const int cnt = act ? g.pl_count[s] : 0;
    const int steps = list_steps(cnt);
    double2 p0 = make_double2(0, 0), p1 = p0, p2 = p0, p3 = p0, p4 = p0, p5 = p0, p6 = p0, p7 = p0;
    if (act) {
        const double2 *ra = rec2(rec, s);
        p0 = ra[0]; p1 = ra[1]; p2 = ra[2]; p3 = ra[3]; p4 = ra[4]; p5 = ra[5]; p6 = ra[6]; p7 = ra[7];
    }
    const double xa = p0.x, ya = p0.y, za = p1.x, vxa = p1.y, vya = p2.x, vza = p2.y;
    const double rho_a = p3.x;
    Acc64 acc;
    if (q == 0) acc.rs = p7.x * k.Wn;  // own term m_a W(0), once
    const double c_a = p7.y;
    const double Ta[6] = {p4.x, p4.y, p5.x, p5.y, p6.x, p6.y};
    const bool tens_a = kExt && signbit(c_a);
    const char *recs = reinterpret_cast<const char *>(rec);
    const int32_t *row = g.pl_slot + base + __lane_id();
    // One step ahead: each lane reads its step-j record into registers, the wavefront
    // syncs, the gathers of step j + kSplit are issued, and step j is evaluated while
    // they are in flight.
    if (q < steps) gather_dma8(recs, kRec * 8, row[(int64_t)q << 6], buf);
    int nxt = q + kSplit < steps ? row[(int64_t)(q + kSplit) << 6] : 0;
    for (int j = q; j < steps; j += kSplit) {
        wait_vm();
        const double2 b0 = dma8_chunk(buf, 0), b1 = dma8_chunk(buf, 1), b2 = dma8_chunk(buf, 2),
                      b3 = dma8_chunk(buf, 3), b4 = dma8_chunk(buf, 4), b5 = dma8_chunk(buf, 5),
                      b6 = dma8_chunk(buf, 6), b7 = dma8_chunk(buf, 7);
        wave_sync();
        if (j + kSplit < steps) {
            gather_dma8(recs, kRec * 8, nxt, buf);
            if (j + 2 * kSplit < steps) nxt = row[(int64_t)(j + 2 * kSplit) << 6];
        }
        if (j < cnt) {
            const double d2 = dist2_exact(xa, ya, za, b0.x, b0.y, b1.x);
            if (d2 < k.h2) {
                const double Tb[6] = {b4.x, b4.y, b5.x, b5.y, b6.x, b6.y};
                pair64<kCorr, kExt>(k, d2, xa - b0.x, ya - b0.y, za - b1.x, b1.y - vxa, b2.x - vya,
                                    b2.y - vza, rho_a, b3.x, p4.x + b4.x, p4.y + b4.y, p5.x + b5.x,
                                    p5.y + b5.y, p6.x + b6.x, p6.y + b6.y, b7.x, b3.y, acc, Ta, Tb,
                                    tens_a, c_a, b7.y);
            }
        }
    }
    fold_acc64<kSplit, kSplit * 64 * 16, kCorr, kExt>(acc, reinterpret_cast<double *>(lbuf));
    if (q != 0 || !act) return;
    postpass(k, io_index(g, s), rho_a, acc.L, acc.ax, acc.ay, acc.az, acc.rs, st, out,
             kCorr ? acc.M : nullptr);
    if (kExt) postpass_ext(k, io_index(g, s), acc, st, out);
    if (Lout) store_vgrad<kCorr>(Lout, s, acc.L, acc.M);
}

// ----------------------------------------- pairs, FP32 + Kahan sums --
// unpacked FP32 record of a partner
struct Src32 {
    double x, y, z;
    float vx, vy, vz, rho, m, V, T[6], c;
};

__device__ inline Src32 src32(double2 c0, double2 c1, double2 c2, double2 c3, double2 c4) {
    Src32 r;
    r.x = c0.x;
    r.y = c0.y;
    r.z = c1.x;
    const float2 a = __builtin_bit_cast(float2, c1.y);
    const float4 b = __builtin_bit_cast(float4, c2);
    const float4 t = __builtin_bit_cast(float4, c3);
    const float4 u = __builtin_bit_cast(float4, c4);
    r.vx = a.x; r.vy = a.y; r.vz = b.x; r.rho = b.y; r.m = b.z; r.V = b.w;
    r.T[0] = t.x; r.T[1] = t.y; r.T[2] = t.z; r.T[3] = t.w; r.T[4] = u.x; r.T[5] = u.y;
    r.c = u.z;
    return r;
}

__device__ inline Src32 load32(const float *r32, int64_t s) {
    const double2 *p = reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(r32) +
                                                         s * kRec32Bytes);
    return src32(p[0], p[1], p[2], p[3], p[4]);
}

template <bool kCorr, bool kExt>
__device__ inline void pair32_of(const Consts32 &kf, const Src32 &a, const Src32 &b, double d2,
                                 Acc32 &acc) {
    pair32<kCorr, kExt>(kf, (float)d2, (float)(a.x - b.x), (float)(a.y - b.y),
                        (float)(a.z - b.z), b.vx - a.vx, b.vy - a.vy, b.vz - a.vz, a.rho, b.rho,
                        a.T[0] + b.T[0], a.T[1] + b.T[1], a.T[2] + b.T[2], a.T[3] + b.T[3],
                        a.T[4] + b.T[4], a.T[5] + b.T[5], b.m, b.V, acc, a.T, b.T, a.c, b.c);
}

// the compensated FP32 sums as FP64 values (rs without the particle's own term)
template <bool kCorr, bool kExt>
__device__ inline Acc64 sums_of(const Acc32 &acc) {
    Acc64 v;
    v.rs = acc.rs.value();
#pragma unroll
    for (int c = 0; c < 9; ++c) v.L[c] = acc.L[c].value();
    v.ax = acc.ax.value();
    v.ay = acc.ay.value();
    v.az = acc.az.value();
    if constexpr (kCorr) {
#pragma unroll
        for (int c = 0; c < 6; ++c) v.M[c] = acc.M[c].value();
    }
    if constexpr (kExt) {
        v.du = acc.du.value();
#pragma unroll
        for (int c = 0; c < 3; ++c) v.xs[c] = acc.xs[c].value();
    }
    return v;
}

template <bool kCorr, bool kExt>
__device__ inline void post32(const Consts &k, int a, double rho_a, double m_a, const Acc64 &acc,
                              const StateDev &st, const OutDev &out, double *Lout, int64_t n,
                              int64_t s) {
    if constexpr (kExt) {
        if (out.du) out.du[a] = 0.5 * acc.du;
        if (out.dx) {
            out.dx[a] = st.vx[a] + k.xsph * acc.xs[0];
            out.dy[a] = st.vy[a] + k.xsph * acc.xs[1];
            out.dz[a] = st.vz[a] + k.xsph * acc.xs[2];
        }
    }
    const double rs = m_a * k.Wn + acc.rs;
    postpass(k, a, rho_a, acc.L, acc.ax, acc.ay, acc.az, rs, st, out, kCorr ? acc.M : nullptr);
    if (Lout) store_vgrad<kCorr>(Lout, s, acc.L, acc.M);
}

template <bool kCorr, bool kExt>
__global__ __launch_bounds__(kBlock) void k_pairs32(GridDev g, int64_t n, Consts k,
                                                    const double *__restrict__ rec,
                                                    const float *__restrict__ r32, StateDev st,
                                                    OutDev out, double *__restrict__ Lout) {
    const int64_t s = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (s >= n) return;
    const Src32 a = load32(r32, s);
    const double2 p3 = rec2(rec, s)[3], p7 = rec2(rec, s)[7];
    const Consts32 kf = narrow(k);
    Acc32 acc;
    for_each_candidate(g, s, a.x, a.y, a.z, k.reach, [&](int t) {
        const Src32 b = load32(r32, t);
        const double d2 = dist2_exact(a.x, a.y, a.z, b.x, b.y, b.z);
        if (d2 < k.h2) pair32_of<kCorr, kExt>(kf, a, b, d2, acc);
    });
    post32<kCorr, kExt>(k, io_index(g, s), p3.x, p7.x, sums_of<kCorr, kExt>(acc), st, out, Lout, n,
                        s);
}

// FP32 pair sums over the frozen pair list (cooperative gathers of the 80-byte records)
// the FP32 form over the frozen pair list, kSplit wavefronts per block of 64 slots as
// in the FP64 list kernel (each wavefront's compensated sums folded as FP64 values)
template <bool kCorr, bool kExt>
__global__ __launch_bounds__(64 * kSplit) void k_pairs32_list(GridDev g, int64_t n, Consts k,
                                                              const double *__restrict__ rec,
                                                              const float *__restrict__ r32,
                                                              StateDev st, OutDev out,
                                                              double *__restrict__ Lout) {
    __shared__ double2 lbuf[kSplit][64 * 5];
    const int q = threadIdx.x >> 6;
    double2 *buf = lbuf[q];
    const int64_t w = xcd_block(gridDim.x);
    const int64_t w0 = w * 64;
    if (w0 >= n) return;  // whole workgroup past the end
    const int64_t s = w0 + __lane_id();
    const bool act = s < n;
    const int64_t base = g.pl_block[w];
    const int cnt = act ? g.pl_count[s] : 0;
    const int steps = list_steps(cnt);
    const Src32 a = load32(r32, act ? s : w0);
    const Consts32 kf = narrow(k);
    Acc32 acc;
    const char *recs = reinterpret_cast<const char *>(r32);
    const int32_t *row = g.pl_slot + base + __lane_id();
    // one step ahead, as in the FP64 kernel
    if (q < steps) gather_dma<5>(recs, kRec32Bytes, row[(int64_t)q << 6], buf);
    int nxt = q + kSplit < steps ? row[(int64_t)(q + kSplit) << 6] : 0;
    for (int j = q; j < steps; j += kSplit) {
        wait_vm();
        const Src32 b = src32(dma_chunk<5>(buf, 0), dma_chunk<5>(buf, 1), dma_chunk<5>(buf, 2),
                              dma_chunk<5>(buf, 3), dma_chunk<5>(buf, 4));
        wave_sync();
        if (j + kSplit < steps) {
            gather_dma<5>(recs, kRec32Bytes, nxt, buf);
            if (j + 2 * kSplit < steps) nxt = row[(int64_t)(j + 2 * kSplit) << 6];
        }
        if (j < cnt) {
            const double d2 = dist2_exact(a.x, a.y, a.z, b.x, b.y, b.z);
            if (d2 < k.h2) pair32_of<kCorr, kExt>(kf, a, b, d2, acc);
        }
    }
    Acc64 sums = sums_of<kCorr, kExt>(acc);
    fold_acc64<kSplit, kSplit * 64 * 5 * 2, kCorr, kExt>(sums, reinterpret_cast<double *>(lbuf));
    if (q != 0 || !act) return;
    const double2 p3 = rec2(rec, s)[3], p7 = rec2(rec, s)[7];
    post32<kCorr, kExt>(k, io_index(g, s), p3.x, p7.x, sums, st, out, Lout, n, s);
}

}  // namespace

int invert_launch(const GridDev &g, int64_t n, int32_t *inv, hipStream_t s) {
    if (!g.io) return SPH_OK;
    k_invert<<<blocks_for(n), kBlock, 0, s>>>(g.io, n, inv);
    SPH_LAUNCHED();
    return SPH_OK;
}

int prepass_launch(const GridDev &g, const StateDev &st, int64_t n, const Consts &k, double *rec,
                   int32_t *status, hipStream_t s, const OutDev *od, int32_t *inv) {
    if (g.io && inv) {
        k_invert<<<blocks_for(n), kBlock, 0, s>>>(g.io, n, inv);
        SPH_LAUNCHED();
    } else {
        inv = nullptr;
    }
    k_prepass<<<blocks_for(n), kBlock, 0, s>>>(g, st, n, k, rec, status, od ? od->dd3 : nullptr,
                                               od ? od->n_act : nullptr, inv);
    SPH_LAUNCHED();
    return SPH_OK;
}

size_t rhs_ws_bytes(int64_t n) {
    Carve c(nullptr);
    c.take<double>((size_t)n * kRec);
    c.take<float>((size_t)n * kRec32);
    c.take<int32_t>(n);
    return c.used;
}

int check_state(const sph_grid *grid, const sph_state *st) {
    if (!st) return fail(SPH_ERR_INVALID_ARG, "state is NULL");
    if (st->n != grid->n) return fail(SPH_ERR_INVALID_ARG, "state n differs from grid n");
    const double *p[] = {st->x,   st->y,   st->z,   st->vx,  st->vy,  st->vz,  st->rho,
                         st->sxx, st->syy, st->szz, st->sxy, st->sxz, st->syz, st->m};
    for (const double *q : p)
        if (!q) return fail(SPH_ERR_INVALID_ARG, "state array is NULL");
    if (!st->flaw_ptr != !st->flaw_eps)
        return fail(SPH_ERR_INVALID_ARG, "flaw_ptr and flaw_eps are given together or not at all");
    return SPH_OK;
}

int check_params(const sph_grid *grid, const sph_params *pr) {
    if (!pr) return fail(SPH_ERR_INVALID_ARG, "params is NULL");
    const double v[] = {pr->h,       pr->rho0,   pr->c,     pr->mu,      pr->Y0,    pr->alpha,
                        pr->beta,    pr->eps_v,  pr->rho_cut, pr->correction, pr->eps_s, pr->n_s,
                        pr->dmpd,    pr->xsph,   pr->eos,   pr->n_M,     pr->a_T,   pr->b_T,
                        pr->A_T,     pr->B_T,    pr->E0_T,  pr->alpha_T, pr->beta_T, pr->E_iv,
                        pr->E_cv};
    for (double q : v)
        if (!std::isfinite(q)) return fail(SPH_ERR_INVALID_ARG, "non-finite parameter");
    if (!(pr->h > 0.0) || !(pr->rho0 > 0.0) || !(pr->c > 0.0))
        return fail(SPH_ERR_INVALID_ARG, "h, rho0 and c must be positive");
    if (pr->mu < 0.0 || !(pr->Y0 > 0.0) || pr->eps_v <= 0.0 || pr->rho_cut < 0.0)
        return fail(SPH_ERR_INVALID_ARG, "mu >= 0, Y0 > 0, eps_v > 0, rho_cut >= 0 required");
    if (pr->h > grid->h) return fail(SPH_ERR_INVALID_ARG, "h exceeds the grid's support radius");
    if (pr->correction != 0.0 && pr->correction != 1.0)
        return fail(SPH_ERR_INVALID_ARG, "correction must be 0 or 1");
    if (pr->eps_s < 0.0 || !(pr->xsph >= 0.0 && pr->xsph <= 1.0))
        return fail(SPH_ERR_INVALID_ARG, "eps_s >= 0 and 0 <= xsph <= 1 required");
    if (pr->eps_s > 0.0 && (!(pr->n_s > 0.0) || !(pr->dmpd > 0.0) || !(pr->dmpd < pr->h)))
        return fail(SPH_ERR_INVALID_ARG, "artificial stress needs n_s > 0 and 0 < dmpd < h");
    if (pr->eos != 0.0 && pr->eos != 1.0 && pr->eos != 2.0)
        return fail(SPH_ERR_INVALID_ARG, "eos must be 0 (liquid), 1 (Murnaghan) or 2 (Tillotson)");
    if (pr->eos == 1.0 && !(pr->n_M > 0.0)) return fail(SPH_ERR_INVALID_ARG, "n_M must be positive");
    if (pr->eos == 2.0 && (!(pr->E0_T > 0.0) || !(pr->E_cv > pr->E_iv) || pr->E_iv < 0.0))
        return fail(SPH_ERR_INVALID_ARG, "Tillotson needs E0_T > 0 and 0 <= E_iv < E_cv");
    return SPH_OK;
}

int check_deriv(const sph_deriv *o) {
    if (!o) return fail(SPH_ERR_INVALID_ARG, "output is NULL");
    const double *p[] = {o->ax, o->ay, o->az, o->drho, o->dsxx, o->dsyy, o->dszz,
                         o->dsxy, o->dsxz, o->dsyz};
    for (const double *q : p)
        if (!q) return fail(SPH_ERR_INVALID_ARG, "output array is NULL");
    if (!(o->dx && o->dy && o->dz) && (o->dx || o->dy || o->dz))
        return fail(SPH_ERR_INVALID_ARG, "dx, dy and dz are given together or not at all");
    if (!o->dd3 != !o->n_act)
        return fail(SPH_ERR_INVALID_ARG, "dd3 and n_act are given together or not at all");
    return SPH_OK;
}

int check_damage(const sph_state *st, const sph_params *pr, const sph_deriv *o) {
    if (o->dd3 && !st->flaw_ptr)
        return fail(SPH_ERR_INVALID_ARG, "damage rates need the flaw lists");
    if (o->dd3 && !(pr->mu > 0.0))
        return fail(SPH_ERR_INVALID_ARG, "damage rates need mu > 0 (Young's modulus)");
    return SPH_OK;
}

// Forward right-hand side on a carved workspace (also used by the leapfrog).
double *rhs_rec_of(Carve c, int64_t n) { return c.take<double>((size_t)n * kRec); }

int rhs_launch(const sph_grid *grid, const sph_state *state, const sph_params *params,
               int precision, const sph_deriv *out, Carve &c, hipStream_t s, double *L_out,
               bool slot_state, bool rec_ready, bool timed) {
    const int64_t n = grid->n;
    GridDev g = grid_dev(grid);
    if (slot_state) g.io = nullptr;
    Consts k = make_consts(*params, g.delta);
    double *rec = rhs_rec_of(c, n);
    c.take<double>((size_t)n * kRec);
    if (out->rec && !rec_ready) rec = out->rec;  // the records go to the caller's buffer
    float *r32 = c.take<float>((size_t)n * kRec32);
    int32_t *inv = c.take<int32_t>(n);
    StateDev st = state_dev(state);
    OutDev od = out_dev(out);
    int rc;
    if (od.dd3 && rec_ready)
        return fail(SPH_ERR_NOT_IMPLEMENTED, "damage rates need the prepass");
    if (!rec_ready && (rc = prepass_launch(g, st, n, k, rec, c.status(), s, &od, inv))) return rc;
    const bool ext = k.eps_s > 0.0 || od.du || od.dx || k.eos != 0;
    if (precision == SPH_FP64) {
        TimedRegion t(timed ? "pairs_fp64" : nullptr, s);
        const dim3 gb(blocks_for(n)), tb(kBlock);
        auto launch = [&](auto corr, auto extra) {
            constexpr bool C = decltype(corr)::value, E = decltype(extra)::value;
            if (g.pl_count)
                k_pairs64_list<C, E><<<blocks_for(n, 64), 64 * kSplit, 0, s>>>(g, n, k, rec, st, od,
                                                                             L_out);
            else
                k_pairs64<C, E><<<gb, tb, 0, s>>>(g, n, k, rec, st, od, L_out);
        };
        using T = std::true_type;
        using F = std::false_type;
        if (k.corr && ext)
            launch(T{}, T{});
        else if (k.corr)
            launch(T{}, F{});
        else if (ext)
            launch(F{}, T{});
        else
            launch(F{}, F{});
        SPH_LAUNCHED();
    } else {
        k_narrow<<<blocks_for(n), kBlock, 0, s>>>(rec, n, r32);
        SPH_LAUNCHED();
        TimedRegion t(timed ? "pairs_fp32comp" : nullptr, s);
        const dim3 gb(blocks_for(n)), tb(kBlock);
        auto launch = [&](auto corr, auto extra) {
            constexpr bool C = decltype(corr)::value, E = decltype(extra)::value;
            if (g.pl_count)
                k_pairs32_list<C, E><<<blocks_for(n, 64), 64 * kSplit, 0, s>>>(g, n, k, rec, r32, st,
                                                                             od, L_out);
            else
                k_pairs32<C, E><<<gb, tb, 0, s>>>(g, n, k, rec, r32, st, od, L_out);
        };
        using T = std::true_type;
        using F = std::false_type;
        if (k.corr && ext)
            launch(T{}, T{});
        else if (k.corr)
            launch(T{}, F{});
        else if (ext)
            launch(F{}, T{});
        else
            launch(F{}, F{});
        SPH_LAUNCHED();
    }
    return SPH_OK;
}

// ------------------------------------------------ the allocation-free variant --
// Scratch of sph_rhs_noalloc: the workspace of sph_rhs for up to kNoallocMaxN
// particles (status word, FP64 operand records, FP32 records), held by every device
// the library runs on until the process ends.
constexpr int64_t kNoallocMaxN = SPH_NOALLOC_MAX_N;
constexpr size_t kNoallocBytes = kAlign + (size_t)kNoallocMaxN * kRec * sizeof(double) +
                                 (size_t)kNoallocMaxN * kRec32 * sizeof(float) +
                                 (size_t)kNoallocMaxN * sizeof(int32_t);
static_assert(kNoallocMaxN % 64 == 0, "record arrays stay 256-byte aligned");
__device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

// Device address of this device's copy of `scratch` (the array's name is only a
// host-side stand-in in host code), looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void **out) {
    int dev = -1;
    SPH_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SPH_ERR_INVALID_ARG, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SPH_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SPH_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPH_OK;
}

__global__ void k_copy_status(const int32_t *__restrict__ from, int32_t *__restrict__ to) { *to = *from; }

}  // namespace

}  // namespace sph

using namespace sph;

extern "C" int sph_rhs_noalloc(const sph_grid *grid, const sph_state *state,
                               const sph_params *params, int precision, const sph_deriv *out,
                               int32_t *status, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_state(grid, state)) ||
        (rc = check_params(grid, params)) || (rc = check_deriv(out)) ||
        (rc = check_damage(state, params, out)))
        return rc;
    if (precision != SPH_FP64 && precision != SPH_FP32_COMP)
        return fail(SPH_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (out->vgrad && precision != SPH_FP64)
        return fail(SPH_ERR_INVALID_ARG, "vgrad is written by the FP64 form only");
    if (grid->n > kNoallocMaxN)
        return fail(SPH_ERR_CAPACITY, "sph_rhs_noalloc serves at most %lld particles (%lld given)",
                    (long long)kNoallocMaxN, (long long)grid->n);
    if (rhs_ws_bytes(grid->n) > kNoallocBytes)
        return fail(SPH_ERR_CAPACITY, "scratch smaller than the workspace of %lld particles",
                    (long long)grid->n);
    void *ws = nullptr;
    if ((rc = scratch_of_current_device(&ws))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = clear_status(ws, s))) return rc;
    Carve c(ws);
    if ((rc = rhs_launch(grid, state, params, precision, out, c, s, out->vgrad, false, false, false)))
        return rc;
    if (status) {
        k_copy_status<<<1, 1, 0, s>>>(reinterpret_cast<const int32_t *>(ws), status);
        SPH_LAUNCHED();
    }
    return SPH_OK;
}

extern "C" int sph_rhs(const sph_grid *grid, const sph_state *state, const sph_params *params,
                       int precision, const sph_deriv *out, void *ws, size_t ws_bytes,
                       void *stream) {
    clear_error();
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_state(grid, state)) ||
        (rc = check_params(grid, params)) || (rc = check_deriv(out)) ||
        (rc = check_damage(state, params, out)))
        return rc;
    if (precision != SPH_FP64 && precision != SPH_FP32_COMP)
        return fail(SPH_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (out->vgrad && precision != SPH_FP64)
        return fail(SPH_ERR_INVALID_ARG, "vgrad is written by the FP64 form only");
    if (!ws) return fail(SPH_ERR_INVALID_ARG, "workspace is NULL");
    const size_t need = rhs_ws_bytes(grid->n);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = clear_status(ws, s))) return rc;
    Carve c(ws);
    return rhs_launch(grid, state, params, precision, out, c, s, out->vgrad);
}
