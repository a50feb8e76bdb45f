// Per-particle and per-pair arithmetic of the right-hand side, shared by the
// forward kernels, the adjoint and the leapfrog.
#pragma once

#include "common.hpp"

namespace sph {

struct Consts {
    double h, h2, inv_h, reach;
    double Wn;  // s / h^3
    double Fn;  // 6 s / h^5
    double rho0, c2, mu, Y0, Y0sq;
    double alpha_c, beta, epsh2, rho_cut;
    int corr;  // correction tensor of section 3.1.6 on the stress-rate gradient
    // artificial stress (section 3.1.4): eps_s, exponent, 1 / w(dmpd / h); XSPH factor
    double eps_s, n_s, inv_wm, xsph;
    int n_int;  // the exponent when it is a whole number in 1..16 (powers by multiplication), else 0
    // equation of state: 0 liquid, 1 Murnaghan (n_M, K0 = rho0 c^2), 2 Tillotson
    int eos;
    double alpha, c, n_M, K0, aT, bT, AT, BT, E0T, alT, beT, Eiv, Ecv;
    // damage model (section 3.2): bulk modulus K (rho0 c^2, A_T for Tillotson) and
    // Young's modulus E = 9 K mu / (3 K + mu)
    double Kd, Ey;
};

// Kernel shape w(q) of section 3.1.1 (W = s/h^3 w), host side.
inline double kernel_shape(double q) {
    if (q < 0.5) return 1.0 + 6.0 * q * q * (q - 1.0);
    if (q < 1.0) return 2.0 * (1.0 - q) * (1.0 - q) * (1.0 - q);
    return 0.0;
}

inline Consts make_consts(const sph_params &p, double delta) {
    Consts k;
    k.h = p.h;
    k.h2 = p.h * p.h;
    k.inv_h = 1.0 / p.h;
    k.reach = (p.h + delta) * (1.0 + 1e-9);
    const double h3 = p.h * p.h * p.h;
    k.Wn = kSigma3 / h3;
    k.Fn = 6.0 * kSigma3 / (h3 * p.h * p.h);
    k.rho0 = p.rho0;
    k.c2 = p.c * p.c;
    k.mu = p.mu;
    k.Y0 = p.Y0;
    k.Y0sq = p.Y0 * p.Y0;
    k.alpha_c = p.alpha * p.c;
    k.beta = p.beta;
    k.epsh2 = p.eps_v * p.h * p.h;
    k.rho_cut = p.rho_cut;
    k.corr = p.correction != 0.0;
    k.eps_s = p.eps_s;
    k.n_s = p.n_s;
    k.inv_wm = p.eps_s > 0.0 ? 1.0 / kernel_shape(p.dmpd / p.h) : 0.0;
    k.xsph = p.xsph;
    k.n_int = (p.n_s >= 1.0 && p.n_s <= 16.0 && p.n_s == (double)(int)p.n_s) ? (int)p.n_s : 0;
    k.eos = (int)p.eos;
    k.alpha = p.alpha;
    k.c = p.c;
    k.n_M = p.n_M;
    k.K0 = p.rho0 * p.c * p.c;
    k.aT = p.a_T;
    k.bT = p.b_T;
    k.AT = p.A_T;
    k.BT = p.B_T;
    k.E0T = p.E0_T;
    k.alT = p.alpha_T;
    k.beT = p.beta_T;
    k.Eiv = p.E_iv;
    k.Ecv = p.E_cv;
    k.Kd = k.eos == 2 ? p.A_T : k.K0;
    k.Ey = 9.0 * k.Kd * p.mu / (3.0 * k.Kd + p.mu);
    return k;
}

struct Consts32 {
    float inv_h, Wn, Fn, h, alpha_c, beta, epsh2;
    float alpha, eps_s, inv_wm, n_s;  // the extended terms (see Consts)
    int n_int;
};

__host__ __device__ inline Consts32 narrow(const Consts &k) {
    return Consts32{(float)k.inv_h, (float)k.Wn,    (float)k.Fn,     (float)k.h,
                    (float)k.alpha_c, (float)k.beta, (float)k.epsh2, (float)k.alpha,
                    (float)k.eps_s, (float)k.inv_wm, (float)k.n_s,   k.n_int};
}

struct StateDev {
    const double *x, *y, *z, *vx, *vy, *vz, *rho, *sxx, *syy, *szz, *sxy, *sxz, *syz, *m;
    const double *u;  // specific internal energy (Tillotson), null = 0
    const double *d;  // damage, null = 0
    const int64_t *fp;  // flaw lists: offsets (n + 1) and ascending thresholds
    const double *fe;
};

inline StateDev state_dev(const sph_state *s) {
    return StateDev{s->x,   s->y,   s->z,   s->vx,  s->vy,  s->vz,  s->rho, s->sxx,
                    s->syy, s->szz, s->sxy, s->sxz, s->syz, s->m,   s->u,   s->d,
                    s->flaw_ptr, s->flaw_eps};
}

struct OutDev {
    double *ax, *ay, *az, *drho, *dsxx, *dsyy, *dszz, *dsxy, *dsxz, *dsyz, *rho_sum;
    double *du, *dx, *dy, *dz;  // energy rate and dx/dt (null unless requested)
    double *dd3;                // damage rate d(d^(1/3))/dt and activated flaws (idem)
    int32_t *n_act;
};

inline OutDev out_dev(const sph_deriv *o) {
    return OutDev{o->ax,   o->ay,   o->az,   o->drho, o->dsxx,    o->dsyy, o->dszz, o->dsxy,
                  o->dsxz, o->dsyz, o->rho_sum, o->du, o->dx, o->dy, o->dz, o->dd3, o->n_act};
}

// Slot-ordered operand records, one 128-byte record per slot:
//   x y z vx | vy vz rho V | T0 T1 T2 T3 | T4 T5 m c
// with T = sigma / rho^2 (xx, yy, zz, xy, xz, yz), V = m / rho and c the sound
// speed, negated (sign bit set, also for 0) when the pressure is negative: the
// artificial stress's tension test.  A partner's
// first seven 16-byte chunks carry everything its pair terms need (its mass being
// V rho), which the adjoint's gathers use; the forward kernels read all eight (the
// eighth also holds the sound speed c, which other equations of state than the
// liquid one vary per particle).
constexpr int kRec = 16;
// FP32 record, 80 bytes per slot: FP64 position (for the exact partner test and
// the differences) and the FP32 operands:
//   x y (f64) | z (f64) vx vy | vz rho m V | T0 T1 T2 T3 | T4 T5 - -
constexpr int kRec32 = 20;  // in floats
constexpr int kRec32Bytes = 80;

__device__ inline const double2 *rec2(const double *rec, int64_t s) {
    return reinterpret_cast<const double2 *>(rec + s * kRec);
}

__device__ inline const float4 *rec4(const float *r32, int64_t s) {
    return reinterpret_cast<const float4 *>(r32 + s * kRec32);
}

// Orders a wavefront's LDS accesses (writes by some lanes before reads by
// others); no other synchronisation is needed inside one wavefront.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Waits until every vector-memory load of the wavefront has completed (s_waitcnt
// vmcnt(0), other counters untouched): the LDS-direct gathers of a step have landed.
__device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The list kernels give one block of 64 slots to a workgroup of P wavefronts: wavefront
// q evaluates the block's list steps q, q + P, q + 2P, ... for the same 64 targets.  So a
// launch holds P times fewer slots in flight per XCD for the same number of wavefronts,
// and the partner records those slots gather stay in that XCD's L2.  fold_waves then
// adds the P partial sums of each target into wavefront 0 in wavefront order (bit
// reproducible): wavefronts 1 .. P-1 store their F values per lane in LDS (scratch, Cap
// doubles, in rounds of Cap / (64 (P - 1)) values), wavefront 0 adds them.  Every thread
// of the workgroup calls it; it starts with a workgroup barrier, so scratch may alias
// buffers that the wavefronts read before the call.
// Steps of a block of the pair list: the longest of its 64 lists (each lane holding
// its slot's count, 0 past the end).
__device__ inline int list_steps(int cnt) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt = max(cnt, __shfl_xor(cnt, o));
    return __builtin_amdgcn_readfirstlane(cnt);
}

constexpr int kSplit = 4;     // wavefronts per block in the forward list kernels
constexpr int kSplitAdj = 4;  // and in the adjoint's pair kernel

template <int P, int Cap, int F>
__device__ inline void fold_waves(double (&v)[F], double *scratch) {
    static_assert(P >= 2 && Cap >= 64 * (P - 1), "scratch too small");
    constexpr int G = Cap / (64 * (P - 1));  // values per round
    const int q = threadIdx.x >> 6, lane = __lane_id();
#pragma unroll
    for (int f0 = 0; f0 < F; f0 += G) {
        __syncthreads();
        if (q > 0) {
#pragma unroll
            for (int f = f0; f < (f0 + G < F ? f0 + G : F); ++f)
                scratch[((q - 1) * G + (f - f0)) * 64 + lane] = v[f];
        }
        __syncthreads();
        if (q == 0) {
#pragma unroll
            for (int r = 1; r < P; ++r)
#pragma unroll
                for (int f = f0; f < (f0 + G < F ? f0 + G : F); ++f)
                    v[f] += scratch[((r - 1) * G + (f - f0)) * 64 + lane];
        }
    }
}

// Coalesced gather of the first N 16-byte chunks of one partner record per lane
// into the wavefront's LDS buffer (64 N chunks).  Each lane holds its list entry of
// the step (one coalesced load by the caller); lane shuffles hand the entries to
// the lanes that load the records' chunks, so that each load instruction moves
// whole records (about eight 128-byte lines) instead of one chunk of 64 scattered
// records.  The loads write LDS themselves (global_load_lds_dwordx4, 1 KB per
// instruction, no registers and no LDS stores): instruction i fills positions
// 64 i .. 64 i + 63, position q holding chunk q % N of record q / N, so record r's
// chunk c sits at buf[N r + c] (an odd N keeps the per-lane reads free of bank
// conflicts).  Every list entry is a valid slot (padding repeats a slot), so no
// load is guarded; lanes ignore the records of their padding entries.  The
// compiler waits for the loads before the first LDS read.
template <int N>
__device__ inline void gather_dma(const char *__restrict__ recs, int stride, int entry,
                                  double2 *buf) {
    static_assert(N % 2 == 1, "odd chunk counts avoid LDS bank conflicts");
    const int lane = __lane_id();
    uint32_t t[N];
#pragma unroll
    for (int i = 0; i < N; ++i)
        t[i] = (uint32_t)__builtin_amdgcn_ds_bpermute(4 * ((64 * i + lane) / N), entry);
    // one barrier for all entries: the shuffles complete together, then the loads issue
    if constexpr (N == 7)
        asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]),
                     "+v"(t[6]));
    else if constexpr (N == 5)
        asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]));
    else
        static_assert(N == 5 || N == 7, "gather widths in use");
    uint32_t st = (uint32_t)stride;
    asm("" : "+s"(st));
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int c = (64 * i + lane) % N;
        __builtin_amdgcn_global_load_lds(
            reinterpret_cast<const void *>(recs + (uint64_t)t[i] * st + c * 16),
            (__attribute__((address_space(3))) void *)(buf + 64 * i), 16, 0, 0);
    }
}

// All eight chunks of 128-byte records, eight whole records (cache lines) per
// instruction: instruction i loads records r = 8 i + (lane >> 3), chunk c landing
// at buf[8 r + ((c + r) & 7)], a rotation that keeps the per-lane reads free of bank
// conflicts.  (Seven chunks per record spread one instruction over ten lines,
// which costs the forward kernel more than the eighth chunk's bytes.)
__device__ inline void gather_dma8(const char *__restrict__ recs, int stride, int entry,
                                   double2 *buf) {
    const int lane = __lane_id();
    const int r0 = lane >> 3;
    const int cc = ((lane & 7) - r0) & 7;
    const char *p = recs + cc * 16;
    const int src = r0 * 4;
    uint32_t t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = (uint32_t)__builtin_amdgcn_ds_bpermute(src + 32 * i, entry);
    asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]),
                 "+v"(t[6]), "+v"(t[7]));
    uint32_t st = (uint32_t)stride;
    asm("" : "+s"(st));
#pragma unroll
    for (int i = 0; i < 8; ++i)
        __builtin_amdgcn_global_load_lds(
            reinterpret_cast<const void *>(p + (uint64_t)t[i] * st),
            (__attribute__((address_space(3))) void *)(buf + 64 * i), 16, 0, 0);
}

// The first four chunks of 128-byte records (position, velocity, density and V),
// sixteen records per instruction: instruction i loads records r = 16 i + (lane >> 2),
// chunk c landing at buf[4 r + ((c + (r >> 2)) & 3)], a rotation that keeps the
// per-lane reads of one chunk free of bank conflicts.
__device__ inline void gather_dma4(const char *__restrict__ recs, int stride, int entry,
                                   double2 *buf) {
    const int lane = __lane_id();
    const int r0 = lane >> 2;
    const int cc = ((lane & 3) - (r0 >> 2)) & 3;  // chunk this lane loads (r >> 2 = r0 >> 2 + 4 i)
    const char *p = recs + cc * 16;
    const int src = r0 * 4;
    uint32_t t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = (uint32_t)__builtin_amdgcn_ds_bpermute(src + 64 * i, entry);
    asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]));
    uint32_t st = (uint32_t)stride;
    asm("" : "+s"(st));
#pragma unroll
    for (int i = 0; i < 4; ++i)
        __builtin_amdgcn_global_load_lds(
            reinterpret_cast<const void *>(p + (uint64_t)t[i] * st),
            (__attribute__((address_space(3))) void *)(buf + 64 * i), 16, 0, 0);
}

__device__ inline double2 dma4_chunk(const double2 *buf, int c) {
    const int L = __lane_id();
    return buf[4 * L + ((c + (L >> 2)) & 3)];
}

__device__ inline double2 dma8_chunk(const double2 *buf, int c) {
    const int L = __lane_id();
    return buf[8 * L + ((c + L) & 7)];
}

// chunk c of this lane's record in a gather_dma<N> buffer
template <int N>
__device__ inline double2 dma_chunk(const double2 *buf, int c) {
    return buf[N * __lane_id() + c];
}

// Liquid equation of state with the optional tension cut-off (section 2.5.1).
__device__ inline double pressure(const Consts &k, double rho) {
    double p = k.c2 * (rho - k.rho0);
    if (k.rho_cut > 0.0 && rho / k.rho0 < k.rho_cut) p = 0.0;
    return p;
}

// Tillotson pressure (section 2.5.3) of one form with its partial derivatives in rho
// and u.  Compressed form: p = (a + b / w) rho u + A chi + B chi^2, w = 1 + u /
// (E0 eta^2); expanded form: p = a rho u + (b rho u / w + A chi e^{-beta z})
// e^{-alpha z^2}, z = rho0 / rho - 1.
// First-order jet in two variables (value and partials along rho and u): evaluating
// the Tillotson forms, which already carry dp/drho and dp/du, on jets gives their
// second partials too, which the adjoint of the sound speed needs.
struct Jet {
    double v, r, u;
};
__device__ inline Jet operator+(Jet a, Jet b) { return {a.v + b.v, a.r + b.r, a.u + b.u}; }
__device__ inline Jet operator-(Jet a, Jet b) { return {a.v - b.v, a.r - b.r, a.u - b.u}; }
__device__ inline Jet operator-(Jet a) { return {-a.v, -a.r, -a.u}; }
__device__ inline Jet operator*(Jet a, Jet b) {
    return {a.v * b.v, a.r * b.v + a.v * b.r, a.u * b.v + a.v * b.u};
}
__device__ inline Jet operator/(Jet a, Jet b) {
    const double i = 1.0 / b.v, q = a.v * i;
    return {q, (a.r - q * b.r) * i, (a.u - q * b.u) * i};
}
__device__ inline Jet operator+(double a, Jet b) { return {a + b.v, b.r, b.u}; }
__device__ inline Jet operator+(Jet a, double b) { return {a.v + b, a.r, a.u}; }
__device__ inline Jet operator-(double a, Jet b) { return {a - b.v, -b.r, -b.u}; }
__device__ inline Jet operator-(Jet a, double b) { return {a.v - b, a.r, a.u}; }
__device__ inline Jet operator*(double a, Jet b) { return {a * b.v, a * b.r, a * b.u}; }
__device__ inline Jet operator*(Jet a, double b) { return {a.v * b, a.r * b, a.u * b}; }
__device__ inline Jet operator/(Jet a, double b) { return a * (1.0 / b); }
__device__ inline Jet operator/(double a, Jet b) {
    const double i = 1.0 / b.v, q = a * i;
    return {q, -q * b.r * i, -q * b.u * i};
}
__device__ inline double ex(double x) { return exp(x); }
__device__ inline Jet ex(Jet x) {
    const double e = exp(x.v);
    return {e, e * x.r, e * x.u};
}
__device__ inline double val(double x) { return x; }
__device__ inline double val(Jet x) { return x.v; }

template <class T>
struct PDerT {
    T p, dr, du;
};
using PDer = PDerT<double>;

// Tillotson pressure (section 2.5.3) of the compressed form, or of the expanded
// one, with its partial derivatives along rho and u
template <class T>
__device__ inline PDerT<T> tillotson_form(const Consts &k, T rho, T u, bool expanded) {
    const T eta = rho / k.rho0, chi = eta - 1.0;
    const T ie2 = 1.0 / (k.E0T * eta * eta);
    const T w = 1.0 + u * ie2;
    const T iw = 1.0 / w;
    const T w_r = -2.0 * u * ie2 / rho;  // dw/drho
    const T g = k.bT * rho * u * iw;     // b rho u / w
    const T g_r = k.bT * u * iw - g * iw * w_r;
    const T g_u = k.bT * rho * iw - g * iw * ie2;
    PDerT<T> d;
    if (!expanded) {
        d.p = k.aT * rho * u + g + k.AT * chi + k.BT * chi * chi;
        d.dr = k.aT * u + g_r + (k.AT + 2.0 * k.BT * chi) / k.rho0;
        d.du = k.aT * rho + g_u;
        return d;
    }
    const T z = k.rho0 / rho - 1.0, z_r = -k.rho0 / (rho * rho);
    const T eb = ex(-k.beT * z), ea = ex(-k.alT * z * z);
    const T q = g + k.AT * chi * eb;
    const T q_r = g_r + k.AT * eb / k.rho0 - k.AT * chi * eb * k.beT * z_r;
    d.p = k.aT * rho * u + q * ea;
    d.dr = k.aT * u + q_r * ea - q * ea * 2.0 * k.alT * z * z_r;
    d.du = k.aT * rho + g_u * ea;
    return d;
}

// Tillotson pressure and partials over its regions: the compressed form for
// rho >= rho0 or u <= E_iv, the expanded form for u >= E_cv, the two joined linearly
// in u between
template <class T>
__device__ inline PDerT<T> tillotson_pd(const Consts &k, T rho, T u) {
    if (val(rho) >= k.rho0 || val(u) <= k.Eiv) return tillotson_form(k, rho, u, false);
    if (val(u) >= k.Ecv) return tillotson_form(k, rho, u, true);
    const PDerT<T> a = tillotson_form(k, rho, u, false), b = tillotson_form(k, rho, u, true);
    const T t = (u - k.Eiv) / (k.Ecv - k.Eiv);
    PDerT<T> d;
    d.p = (1.0 - t) * a.p + t * b.p;
    d.dr = (1.0 - t) * a.dr + t * b.dr;
    d.du = (1.0 - t) * a.du + t * b.du + (b.p - a.p) / (k.Ecv - k.Eiv);
    return d;
}

// Pressure and sound speed of one particle: the liquid equation (above), Murnaghan
// (section 2.5.2) or Tillotson (section 2.5.3, its regions joined linearly in u), the
// sound speed from c^2 = dp/drho|u + p / rho^2 dp/du|rho, at least 0.
__device__ inline void eos_pc(const Consts &k, double rho, double u, double &p, double &cs) {
    if (k.eos == 1) {
        const double eta = rho / k.rho0;
        const double en1 = pow(eta, k.n_M - 1.0);
        p = k.K0 / k.n_M * (en1 * eta - 1.0);
        if (k.rho_cut > 0.0 && eta < k.rho_cut) p = 0.0;
        cs = sqrt(k.K0 / k.rho0 * en1);
    } else if (k.eos == 2) {
        const PDer d = tillotson_pd(k, rho, u);
        p = d.p;
        cs = sqrt(fmax(d.dr + d.p / (rho * rho) * d.du, 0.0));
    } else {
        p = pressure(k, rho);
        cs = k.c;
    }
}

// Second invariant J2 = S:S / 2 of a symmetric stress stored as six components.
__device__ inline double j2_of(const double S[6]) {
    return 0.5 * (S[0] * S[0] + S[1] * S[1] + S[2] * S[2]) + (S[3] * S[3] + S[4] * S[4] + S[5] * S[5]);
}

// von Mises factor f_Y = min(Y0^2 / (3 J2), 1) (section 2.6).
__device__ inline double yield_factor(const Consts &k, const double S[6]) {
    const double j3 = 3.0 * j2_of(S);
    return j3 > k.Y0sq ? k.Y0sq / j3 : 1.0;
}

// Operand record of slot s (pressure, limiter, T = sigma / rho^2, V = m / rho) from
// the particle's state; raises STALE_GRID when the particle left its cell (or its
// list position) by more than skin / 2 and DOMAIN for a non-positive or non-finite
// density, a non-finite velocity or stress, or a damage outside [0, 1].  With damage
// d the stress is sigma_d = -p^ I + (1 - d) f_Y S, p^ = p for p >= 0 and (1 - d) p
// below (section 2.7); d = 0 gives sigma exactly.  Returns the pressure p.  The
// prepass and the leapfrog's fused passes write every record through this one
// function.
__device__ inline double write_rec(const GridDev &g, const Consts &k, int64_t s, double x, double y,
                                   double z, double vx, double vy, double vz, double rho,
                                   const double S[6], double m, double *__restrict__ rec,
                                   int32_t *__restrict__ status, double u = 0.0, double d = 0.0) {
    if (!within_cell(g, (int)s, x, y, z)) raise_flag(status, SPH_ERR_STALE_GRID);
    bool finite = isfinite(rho) && isfinite(vx) && isfinite(vy) && isfinite(vz);
#pragma unroll
    for (int c = 0; c < 6; ++c) finite = finite && isfinite(S[c]);
    if (!(rho > 0.0) || !finite || !(d >= 0.0 && d <= 1.0)) raise_flag(status, SPH_ERR_DOMAIN);
    double p, cs;
    eos_pc(k, rho, u, p, cs);
    const double f = (1.0 - d) * yield_factor(k, S);
    const double ph = p >= 0.0 ? p : (1.0 - d) * p;
    const double ir2 = 1.0 / (rho * rho);
    double2 *r = reinterpret_cast<double2 *>(rec + s * kRec);
    r[0] = make_double2(x, y);
    r[1] = make_double2(z, vx);
    r[2] = make_double2(vy, vz);
    r[3] = make_double2(rho, m / rho);
    r[4] = make_double2((f * S[0] - ph) * ir2, (f * S[1] - ph) * ir2);
    r[5] = make_double2((f * S[2] - ph) * ir2, f * S[3] * ir2);
    r[6] = make_double2(f * S[4] * ir2, f * S[5] * ir2);
    r[7] = make_double2(m, p < 0.0 ? -cs : cs);
    return p;
}

// Largest eigenvalue of a symmetric 3x3 matrix (xx yy zz xy xz yz) by the
// trigonometric solution of its characteristic cubic (O. K. Smith, Commun. ACM 4,
// 1961): with q = tr / 3 and B = (A - q I) / p, p^2 = |A - q I|^2 / 6, the roots are
// q + 2 p cos(acos(det B / 2) / 3 + 2 pi j / 3), the largest at j = 0.
__device__ inline double sym3_max_eig(const double a[6]) {
    const double q = (a[0] + a[1] + a[2]) * (1.0 / 3.0);
    const double b0 = a[0] - q, b1 = a[1] - q, b2 = a[2] - q;
    const double off = a[3] * a[3] + a[4] * a[4] + a[5] * a[5];
    const double p2 = (b0 * b0 + b1 * b1 + b2 * b2 + 2.0 * off) * (1.0 / 6.0);
    if (!(p2 > 0.0)) return q;
    const double pp = sqrt(p2);
    const double det = b0 * (b1 * b2 - a[5] * a[5]) - a[3] * (a[3] * b2 - a[5] * a[4]) +
                       a[4] * (a[3] * a[5] - b1 * a[4]);
    const double r = fmin(fmax(det / (2.0 * p2 * pp), -1.0), 1.0);
    return q + 2.0 * pp * cos(acos(r) * (1.0 / 3.0));
}

// Damage model of section 3.2 for one particle (a: user index): the strain
// eps = sigma_max / ((1 - d) E) from the damaged stress sig (infinite at d = 1), the
// number of the particle's flaw thresholds below it, and the growth rate
// n_act c_g / R_s of d^(1/3), zero once d n_tot >= n_act (the limiter).  Flaw
// offsets that are not ordered within [0, fp[n]] raise DOMAIN and count no flaw.
__device__ inline void damage_rate(const Consts &k, const StateDev &st, int64_t n, int a,
                                   const double sig[6], double rho, double m, double d,
                                   double *dd3, int32_t *nact, int32_t *__restrict__ status) {
    const int64_t lo = st.fp[a], hi = st.fp[a + 1], end = st.fp[n];
    if (lo < 0 || hi < lo || hi > end) {
        raise_flag(status, SPH_ERR_DOMAIN);
        dd3[a] = 0.0;
        nact[a] = 0;
        return;
    }
    const double smax = sym3_max_eig(sig);
    const double eps = d < 1.0 ? smax / ((1.0 - d) * k.Ey) : INFINITY;
    int64_t l = lo, r = hi;  // first threshold >= eps
    while (l < r) {
        const int64_t mid = l + ((r - l) >> 1);
        if (st.fe[mid] < eps)
            l = mid + 1;
        else
            r = mid;
    }
    const int32_t na = (int32_t)(l - lo);
    const double cg = 0.4 * sqrt((k.Kd + 4.0 / 3.0 * (1.0 - d) * k.mu) / rho);
    const double Rs = cbrt(3.0 * m / (4.0 * M_PI * rho));
    const double ntot = (double)(hi - lo);
    dd3[a] = d * ntot < (double)na ? na * cg / Rs : 0.0;
    nact[a] = na;
}

// 1/sqrt(x): hardware estimate refined by two Newton steps y <- y (3 - x y^2) / 2
// (full double precision); +inf at 0.
__device__ inline double rsqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    y = y * fma(-hx, y * y, 1.5);
    return y;
}

// 1/x: hardware estimate refined by two Newton steps y <- y (2 - x y).
__device__ inline double rcp64(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Kernel pieces at distance r (section 3.1.1), branch free: w(q) with
// W = Wn w, and f(q) with W'(r)/r = Fn f; ir = 1/r (+inf at r = 0, where the
// inner piece is selected).
struct KernelPieces {
    double q, w, f;
    bool inner;
};

__device__ inline KernelPieces kernel_pieces(const Consts &k, double d2, double ir) {
    KernelPieces p;
    p.q = d2 > 0.0 ? d2 * ir * k.inv_h : 0.0;
    const double q = p.q;
    const double u = 1.0 - q, u2 = u * u;
    const double w_in = fma(q * q, fma(6.0, q, -6.0), 1.0);
    const double f_in = fma(3.0, q, -2.0);
    const double w_out = 2.0 * u2 * u;
    const double f_out = -u2 * (k.h * ir);  // -(1-q)^2 / q
    p.inner = q < 0.5;
    p.w = p.inner ? w_in : w_out;
    p.f = p.inner ? f_in : f_out;
    return p;
}

// Artificial viscosity Pi*_ab (section 3.1.3) for w = (v_a - v_b).(x_a - x_b):
// nu = h w / (r^2 + eps h^2), Pi = (-alpha c nu + beta nu^2) / ((rho_a + rho_b)/2)
// when w < 0, else 0.  One reciprocal serves both divisions.
struct Visc {
    double Pi, nu, invD, coef;
};

__device__ inline Visc viscosity(const Consts &k, double d2, double w, double ra, double rb,
                                 double alpha_c) {
    Visc v;
    const double D = d2 + k.epsh2, S = ra + rb;
    const double inv = rcp64(D * S);
    v.invD = S * inv;        // 1 / D
    v.coef = 2.0 * D * inv;  // 2 / (rho_a + rho_b)
    v.nu = k.h * w * v.invD;
    const double Pi = (-alpha_c * v.nu + k.beta * v.nu * v.nu) * v.coef;
    v.Pi = w < 0.0 ? Pi : 0.0;
    return v;
}

struct Acc64 {
    double rs = 0.0;
    double L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double ax = 0.0, ay = 0.0, az = 0.0;
    // with the correction: M = sum_b V_b (x_b - x_a) (x) grad_a W_ab, which is
    // -V_b F r r^T per pair and so symmetric (xx yy zz xy xz yz)
    double M[6] = {0, 0, 0, 0, 0, 0};
    // with the extra terms: energy sum (twice du/dt) and XSPH velocity sum
    double du = 0.0, xs[3] = {0, 0, 0};
};

// The sums of the P wavefronts of a list kernel's workgroup added into wavefront 0
// (fold_waves); the correction's and the extra terms' sums only where they are formed.
template <int P, int Cap, bool kCorr, bool kExt>
__device__ inline void fold_acc64(Acc64 &a, double *scratch) {
    constexpr int F = 13 + (kCorr ? 6 : 0) + (kExt ? 4 : 0);
    double v[F];
    int i = 0;
    v[i++] = a.rs;
#pragma unroll
    for (int c = 0; c < 9; ++c) v[i++] = a.L[c];
    v[i++] = a.ax;
    v[i++] = a.ay;
    v[i++] = a.az;
    if constexpr (kCorr) {
#pragma unroll
        for (int c = 0; c < 6; ++c) v[i++] = a.M[c];
    }
    if constexpr (kExt) {
        v[i++] = a.du;
#pragma unroll
        for (int c = 0; c < 3; ++c) v[i++] = a.xs[c];
    }
    fold_waves<P, Cap>(v, scratch);
    i = 0;
    a.rs = v[i++];
#pragma unroll
    for (int c = 0; c < 9; ++c) a.L[c] = v[i++];
    a.ax = v[i++];
    a.ay = v[i++];
    a.az = v[i++];
    if constexpr (kCorr) {
#pragma unroll
        for (int c = 0; c < 6; ++c) a.M[c] = v[i++];
    }
    if constexpr (kExt) {
        a.du = v[i++];
#pragma unroll
        for (int c = 0; c < 3; ++c) a.xs[c] = v[i++];
    }
}

// f^n for a fractional exponent, out of line so that the pair loop does not carry
// the registers of pow
__device__ __attribute__((noinline)) inline double pow_frac(double f, double n) { return pow(f, n); }

// One ordered pair (a target, b partner).  r = x_a - x_b, dv = v_b - v_a,
// B = T_a + T_b (six components).  With kExt also: the artificial stress
// (zeta_a + zeta_b) (w / w(dmpd))^n in the momentum bracket (Ta, Tb: the two
// particles' T, tens_a: a in tension), the energy sum m_b B : dv (x) grad_a W
// (the momentum bracket without artificial stress) and the XSPH sum
// 2 m_b / (rho_a + rho_b) dv W; ca, cb are the records' sound speeds, whose sign
// bit marks tension.
template <bool kCorr = false, bool kExt = false>
__device__ inline void pair64(const Consts &k, double d2, double rx, double ry, double rz,
                              double dvx, double dvy, double dvz, double ra, double rb,
                              double Bxx, double Byy, double Bzz, double Bxy, double Bxz,
                              double Byz, double mb, double Vb, Acc64 &a,
                              const double *Ta = nullptr, const double *Tb = nullptr,
                              bool tens_a = false, double ca = 0.0, double cb = 0.0) {
    const double ir = rsqrt64(d2);
    const KernelPieces kp = kernel_pieces(k, d2, ir);
    const double F = k.Fn * kp.f;
    const double gx = F * rx, gy = F * ry, gz = F * rz;
    a.rs = fma(mb, k.Wn * kp.w, a.rs);
    const double tx = Vb * dvx, ty = Vb * dvy, tz = Vb * dvz;
    a.L[0] = fma(tx, gx, a.L[0]);
    a.L[1] = fma(tx, gy, a.L[1]);
    a.L[2] = fma(tx, gz, a.L[2]);
    a.L[3] = fma(ty, gx, a.L[3]);
    a.L[4] = fma(ty, gy, a.L[4]);
    a.L[5] = fma(ty, gz, a.L[5]);
    a.L[6] = fma(tz, gx, a.L[6]);
    a.L[7] = fma(tz, gy, a.L[7]);
    a.L[8] = fma(tz, gz, a.L[8]);
    const double wab = -(dvx * rx + dvy * ry + dvz * rz);
    // the pair's mean sound speed (section 3.1.3); one value for the liquid equation
    const double Pi =
        viscosity(k, d2, wab, ra, rb, kExt ? k.alpha * (0.5 * (fabs(ca) + fabs(cb))) : k.alpha_c).Pi;
    const double bxx = Bxx - Pi, byy = Byy - Pi, bzz = Bzz - Pi;
    const double qx = bxx * gx + Bxy * gy + Bxz * gz;
    const double qy = Bxy * gx + byy * gy + Byz * gz;
    const double qz = Bxz * gx + Byz * gy + bzz * gz;
    if constexpr (kExt) {
        // energy: B : dv (x) g = dv . (B g)
        a.du = fma(mb, dvx * qx + dvy * qy + dvz * qz, a.du);
        // XSPH
        const double xw = 2.0 * mb * k.Wn * kp.w / (ra + rb);
        a.xs[0] = fma(xw, dvx, a.xs[0]);
        a.xs[1] = fma(xw, dvy, a.xs[1]);
        a.xs[2] = fma(xw, dvz, a.xs[2]);
        // artificial stress
        const bool tens_b = signbit(cb);
        if (k.eps_s > 0.0 && (tens_a || tens_b)) {
            const double f = kp.w * k.inv_wm;
            double fn = f;
            if (k.n_int > 0) {
                for (int e = 1; e < k.n_int; ++e) fn *= f;
            } else {
                fn = pow_frac(f, k.n_s);
            }
            const double za = tens_a ? -k.eps_s : 0.0, zb = tens_b ? -k.eps_s : 0.0;
            double Z[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) Z[i] = (za * Ta[i] + zb * Tb[i]) * fn;
            a.ax = fma(mb, Z[0] * gx + Z[3] * gy + Z[4] * gz, a.ax);
            a.ay = fma(mb, Z[3] * gx + Z[1] * gy + Z[5] * gz, a.ay);
            a.az = fma(mb, Z[4] * gx + Z[5] * gy + Z[2] * gz, a.az);
        }
    }
    a.ax = fma(mb, qx, a.ax);
    a.ay = fma(mb, qy, a.ay);
    a.az = fma(mb, qz, a.az);
    if constexpr (kCorr) {
        const double P = -Vb * F;
        const double px = P * rx, py = P * ry, pz = P * rz;
        a.M[0] = fma(px, rx, a.M[0]);
        a.M[1] = fma(py, ry, a.M[1]);
        a.M[2] = fma(pz, rz, a.M[2]);
        a.M[3] = fma(px, ry, a.M[3]);
        a.M[4] = fma(px, rz, a.M[4]);
        a.M[5] = fma(py, rz, a.M[5]);
    }
}

// Kahan-compensated single-precision sum (Kahan 1965): c carries the low-order
// part lost by the last addition.
struct Kahan {
    float s = 0.0f, c = 0.0f;
    __device__ inline void add(float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ inline double value() const { return (double)s - (double)c; }
};

struct Acc32 {
    Kahan rs, L[9], ax, ay, az, M[6];
    Kahan du, xs[3];  // the extended terms (twice du/dt, XSPH sum)
};

// FP32 form of pair64 (same terms; with kExt the records' sound speeds ca, cb carry
// the tension sign bit, and Ta, Tb are the two particles' T).
template <bool kCorr = false, bool kExt = false>
__device__ inline void pair32(const Consts32 &k, float d2, float rx, float ry, float rz, float dvx,
                              float dvy, float dvz, float ra, float rb, float Bxx, float Byy,
                              float Bzz, float Bxy, float Bxz, float Byz, float mb, float Vb,
                              Acc32 &a, const float *Ta = nullptr, const float *Tb = nullptr,
                              float ca = 0.0f, float cb = 0.0f) {
    const float ir = __builtin_amdgcn_rsqf(d2);
    const float q = d2 > 0.0f ? d2 * ir * k.inv_h : 0.0f;
    const float u = 1.0f - q, u2 = u * u;
    const bool inner = q < 0.5f;
    const float w = inner ? fmaf(q * q, fmaf(6.0f, q, -6.0f), 1.0f) : 2.0f * u2 * u;
    const float f = inner ? fmaf(3.0f, q, -2.0f) : -u2 * (k.h * ir);
    const float F = k.Fn * f;
    const float gx = F * rx, gy = F * ry, gz = F * rz;
    a.rs.add(mb * (k.Wn * w));
    const float tx = Vb * dvx, ty = Vb * dvy, tz = Vb * dvz;
    a.L[0].add(tx * gx);
    a.L[1].add(tx * gy);
    a.L[2].add(tx * gz);
    a.L[3].add(ty * gx);
    a.L[4].add(ty * gy);
    a.L[5].add(ty * gz);
    a.L[6].add(tz * gx);
    a.L[7].add(tz * gy);
    a.L[8].add(tz * gz);
    const float wab = -(dvx * rx + dvy * ry + dvz * rz);
    const float D = d2 + k.epsh2, S = ra + rb;
    const float inv = __builtin_amdgcn_rcpf(D * S);
    const float nu = k.h * wab * S * inv;
    const float alpha_c = kExt ? k.alpha * (0.5f * (fabsf(ca) + fabsf(cb))) : k.alpha_c;
    const float Pi = wab < 0.0f ? (-alpha_c * nu + k.beta * nu * nu) * 2.0f * D * inv : 0.0f;
    const float bxx = Bxx - Pi, byy = Byy - Pi, bzz = Bzz - Pi;
    float qx = bxx * gx + Bxy * gy + Bxz * gz;
    float qy = Bxy * gx + byy * gy + Byz * gz;
    float qz = Bxz * gx + Byz * gy + bzz * gz;
    if constexpr (kExt) {
        a.du.add(mb * (dvx * qx + dvy * qy + dvz * qz));
        const float xw = mb * k.Wn * w * (2.0f * D * inv);  // 2 m_b W / (rho_a + rho_b)
        a.xs[0].add(xw * dvx);
        a.xs[1].add(xw * dvy);
        a.xs[2].add(xw * dvz);
        const bool ta = signbit(ca), tb = signbit(cb);
        if (k.eps_s > 0.0f && (ta || tb)) {
            const float f = w * k.inv_wm;
            float fn = f;
            if (k.n_int > 0) {
                for (int e = 1; e < k.n_int; ++e) fn *= f;
            } else {
                fn = powf(f, k.n_s);
            }
            const float za = ta ? -k.eps_s : 0.0f, zb = tb ? -k.eps_s : 0.0f;
            float Z[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) Z[i] = (za * Ta[i] + zb * Tb[i]) * fn;
            qx += Z[0] * gx + Z[3] * gy + Z[4] * gz;
            qy += Z[3] * gx + Z[1] * gy + Z[5] * gz;
            qz += Z[4] * gx + Z[5] * gy + Z[2] * gz;
        }
    }
    a.ax.add(mb * qx);
    a.ay.add(mb * qy);
    a.az.add(mb * qz);
    if constexpr (kCorr) {
        const float P = -Vb * F;
        const float px = P * rx, py = P * ry, pz = P * rz;
        a.M[0].add(px * rx);
        a.M[1].add(py * ry);
        a.M[2].add(pz * rz);
        a.M[3].add(px * ry);
        a.M[4].add(px * rz);
        a.M[5].add(py * rz);
    }
}

// Correction tensor C = M^{-1} of a symmetric M (xx yy zz xy xz yz) by the
// adjugate, into C[3 i + j]; the identity where det M <= 1e-12 (tr M / 3)^3
// (fewer than three non-coplanar partners) or is not finite, and then false.
// Section 3.1.6.
__device__ inline bool correction_tensor(const double M[6], double C[9]) {
    const double a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5];
    const double A00 = b * c - f * f, A01 = e * f - d * c, A02 = d * f - e * b;
    const double A11 = a * c - e * e, A12 = e * d - a * f, A22 = a * b - d * d;
    const double det = a * A00 + d * A01 + e * A02;
    const double t = (a + b + c) / 3.0;
    if (det > 1e-12 * t * t * t && isfinite(det)) {
        const double id = 1.0 / det;
        C[0] = A00 * id; C[1] = A01 * id; C[2] = A02 * id;
        C[3] = A01 * id; C[4] = A11 * id; C[5] = A12 * id;
        C[6] = A02 * id; C[7] = A12 * id; C[8] = A22 * id;
        return true;
    }
    C[0] = 1.0; C[1] = 0.0; C[2] = 0.0;
    C[3] = 0.0; C[4] = 1.0; C[5] = 0.0;
    C[6] = 0.0; C[7] = 0.0; C[8] = 1.0;
    return false;
}

// Lc = L C (row-major 3x3)
__device__ inline void corrected_gradient(const double L[9], const double M[6], double Lc[9]) {
    double C[9];
    correction_tensor(M, C);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Lc[3 * i + j] = L[3 * i] * C[j] + L[3 * i + 1] * C[3 + j] + L[3 * i + 2] * C[6 + j];
}

// Stress rate (Hooke + Jaumann, section 2.4) and continuity for user particle a
// from its velocity gradient L (L[3 i + j] = dv_i / dx_j), written with the
// other outputs.  S~ = f_Y S;  dS = 2 mu (sym L - tr L / 3 I) + R S~ - S~ R.
// With M (the correction's moment matrix), the strain and rotation rates use
// L C; the continuity equation keeps tr L.
__device__ inline void postpass(const Consts &k, int a, double rho, const double L0[9], double ax,
                                double ay, double az, double rs, const StateDev &st,
                                const OutDev &o, const double *M = nullptr) {
    double S[6] = {st.sxx[a], st.syy[a], st.szz[a], st.sxy[a], st.sxz[a], st.syz[a]};
    const double f = yield_factor(k, S);
    const double sa = f * S[0], sb = f * S[1], sc = f * S[2];
    const double sd = f * S[3], se = f * S[4], sf = f * S[5];
    o.drho[a] = -rho * (L0[0] + L0[4] + L0[8]);
    double Lc[9];
    if (M) {
        corrected_gradient(L0, M, Lc);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) Lc[i] = L0[i];
    }
    const double *L = Lc;
    const double tr = L[0] + L[4] + L[8];
    const double wz = 0.5 * (L[1] - L[3]);  // R_xy
    const double wy = 0.5 * (L[2] - L[6]);  // R_xz
    const double wx = 0.5 * (L[5] - L[7]);  // R_yz
    const double mu2 = 2.0 * k.mu, t3 = tr / 3.0;
    o.dsxx[a] = mu2 * (L[0] - t3) + 2.0 * (wz * sd + wy * se);
    o.dsyy[a] = mu2 * (L[4] - t3) + 2.0 * (wx * sf - wz * sd);
    o.dszz[a] = mu2 * (L[8] - t3) - 2.0 * (wy * se + wx * sf);
    o.dsxy[a] = k.mu * (L[1] + L[3]) + wz * (sb - sa) + wy * sf + wx * se;
    o.dsxz[a] = k.mu * (L[2] + L[6]) + wy * (sc - sa) + wz * sf - wx * sd;
    o.dsyz[a] = k.mu * (L[5] + L[7]) + wx * (sc - sb) - wz * se - wy * sd;
    o.ax[a] = ax;
    o.ay[a] = ay;
    o.az[a] = az;
    if (o.rho_sum) o.rho_sum[a] = rs;
}

// The extra outputs of user particle a: du/dt (eq. energy_sph, half the
// accumulated sum) and dx/dt = v_a + xsph * (XSPH sum).
__device__ inline void postpass_ext(const Consts &k, int a, const Acc64 &acc, const StateDev &st,
                                    const OutDev &o) {
    if (o.du) o.du[a] = 0.5 * acc.du;
    if (o.dx) {
        o.dx[a] = st.vx[a] + k.xsph * acc.xs[0];
        o.dy[a] = st.vy[a] + k.xsph * acc.xs[1];
        o.dz[a] = st.vz[a] + k.xsph * acc.xs[2];
    }
}

// Cotangents of the right-hand side's outputs (user order; null = zero).
struct CotDev {
    const double *ax, *ay, *az, *drho, *ds[6], *rho_sum;
    const double *du, *dx[3];  // energy rate and dx/dt (null = zero)
};

// Gradient destination (user order), overwritten or accumulated.
struct GradDev {
    double *x, *y, *z, *vx, *vy, *vz, *rho, *s[6];
    int accumulate;
    double *u;  // gradient of u (Tillotson), else null
};

// Velocity-gradient handoff (sph_deriv.vgrad) and the adjoint's copy of it: slot s
// holds vgrad_width(corr) values from L[vgrad_width(corr) * s] on: L row by row, then
// with the correction the moment matrix (xx yy zz xy xz yz).
__host__ __device__ constexpr int vgrad_width(bool corr) { return corr ? 15 : 9; }

template <bool kCorr>
__device__ inline void store_vgrad(double *Lout, int64_t s, const double *L, const double *M) {
    double *p = Lout + (size_t)s * vgrad_width(kCorr);
#pragma unroll
    for (int i = 0; i < 9; ++i) p[i] = L[i];
    if constexpr (kCorr) {
#pragma unroll
        for (int i = 0; i < 6; ++i) p[9 + i] = M[i];
    }
}

// adjoint.hip
CotDev cot_dev(const sph_deriv_cot *c);
GradDev grad_dev(const sph_fields *g, int accumulate);
int check_grad(const sph_fields *g);
size_t adjoint_ws_bytes(int64_t n);
// L_in (nullable): the forward velocity gradient of the same state in slot order
// (vgrad_width values per slot); when null it is recomputed.  slot_state: the state, cotangent
// and gradient arrays are in the grid's slot order instead of user order.
// acc_parts (nullable): ceil(n / 256) per-block mu accumulators followed by
// ceil(n / 64) Y0 accumulators (per block, or per wavefront for the list kernel)
// to which the launch adds its sums instead of reducing into dparams.
// post_ready: the operand records and the post stage's outputs (adj_buffers of
// this carve) are already written, with the mu block sums added to acc_parts;
// only the pair stage runs (L_in required).  rec_in (nullable): the operand records
// of the same state that a forward call wrote; the prepass is then not run.
int rhs_adjoint_launch(const sph_grid *grid, const sph_state *state, const sph_params *params,
                       const CotDev &cot, const GradDev &grad, double *dparams, int accumulate_params,
                       Carve &c, hipStream_t s, const double *L_in = nullptr,
                       bool slot_state = false, double *acc_parts = nullptr,
                       bool post_ready = false, const double *rec_in = nullptr);
// dparams[0] (+)= sum of p0[0..m0), dparams[1] (+)= sum of p1[0..m1) (null parts
// skipped), fixed summation order
int reduce_params_launch(const double *p0, int64_t m0, const double *p1, int64_t m1,
                         double *dparams, int accumulate, hipStream_t s);

// rhs.hip
// inv (n int32) := the inverse permutation (slot of every user index), with a
// user-ordered state (g.io set); nothing otherwise
int invert_launch(const GridDev &g, int64_t n, int32_t *inv, hipStream_t s);
// od (nullable): outputs whose dd3 / n_act, when set, receive the damage rates
// inv (nullable): n int32 of scratch; with a user-ordered state the prepass fills it with
// the inverse permutation and reads the state in user order
int prepass_launch(const GridDev &g, const StateDev &st, int64_t n, const Consts &k, double *rec,
                   int32_t *status, hipStream_t s, const OutDev *od = nullptr,
                   int32_t *inv = nullptr);
int check_state(const sph_grid *grid, const sph_state *st);
int check_params(const sph_grid *grid, const sph_params *pr);
int check_deriv(const sph_deriv *o);
// L_out (nullable): the velocity gradient of every slot, 9 arrays of n (slot order),
// followed with the correction by its moment matrix M, 6 arrays (xx yy zz xy xz yz).
// slot_state: the state and output arrays are in the grid's slot order.
// rec_ready: the operand records (the first carve, rhs_rec_of) already hold the
// state's records, so the prepass is skipped.
// timed: bracket the pair kernel for the diagnostic timing table when it is enabled.
int rhs_launch(const sph_grid *grid, const sph_state *state, const sph_params *params,
               int precision, const sph_deriv *out, Carve &c, hipStream_t s,
               double *L_out = nullptr, bool slot_state = false, bool rec_ready = false,
               bool timed = true);
// where rhs_launch on a carve that starts like c keeps its operand records
double *rhs_rec_of(Carve c, int64_t n);
size_t rhs_ws_bytes(int64_t n);

// Deterministic sum over a 256-thread block (fixed tree); every thread must call it.
__device__ inline double block_sum(double v) {
    __shared__ double lds[kBlock];
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) lds[t] += lds[t + off];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

}  // namespace sph
