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
};

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
    return k;
}

struct Consts32 {
    float inv_h, Wn, Fn, h, alpha_c, beta, epsh2;
};

__host__ __device__ inline Consts32 narrow(const Consts &k) {
    return Consts32{(float)k.inv_h, (float)k.Wn, (float)k.Fn, (float)k.h,
                    (float)k.alpha_c, (float)k.beta, (float)k.epsh2};
}

struct StateDev {
    const double *x, *y, *z, *vx, *vy, *vz, *rho, *sxx, *syy, *szz, *sxy, *sxz, *syz, *m;
};

inline StateDev state_dev(const sph_state *s) {
    return StateDev{s->x,   s->y,   s->z,   s->vx,  s->vy,  s->vz,  s->rho,
                    s->sxx, s->syy, s->szz, s->sxy, s->sxz, s->syz, s->m};
}

struct OutDev {
    double *ax, *ay, *az, *drho, *dsxx, *dsyy, *dszz, *dsxy, *dsxz, *dsyz, *rho_sum;
};

inline OutDev out_dev(const sph_deriv *o) {
    return OutDev{o->ax,   o->ay,   o->az,   o->drho, o->dsxx,   o->dsyy,
                  o->dszz, o->dsxy, o->dsxz, o->dsyz, o->rho_sum};
}

// Slot-ordered operands of the pair sums: position, velocity, density,
// T = sigma / rho^2 (xx, yy, zz, xy, xz, yz), mass, V = m / rho.
struct Rec64 {
    double *x, *y, *z, *vx, *vy, *vz, *rho, *t[6], *m, *V;
};

struct Rec32 {
    float *vx, *vy, *vz, *rho, *t[6], *m, *V;
};

inline Rec64 carve_rec64(Carve &c, int64_t n) {
    Rec64 r;
    r.x = c.take<double>(n);
    r.y = c.take<double>(n);
    r.z = c.take<double>(n);
    r.vx = c.take<double>(n);
    r.vy = c.take<double>(n);
    r.vz = c.take<double>(n);
    r.rho = c.take<double>(n);
    for (int i = 0; i < 6; ++i) r.t[i] = c.take<double>(n);
    r.m = c.take<double>(n);
    r.V = c.take<double>(n);
    return r;
}

inline Rec32 carve_rec32(Carve &c, int64_t n) {
    Rec32 r;
    r.vx = c.take<float>(n);
    r.vy = c.take<float>(n);
    r.vz = c.take<float>(n);
    r.rho = c.take<float>(n);
    for (int i = 0; i < 6; ++i) r.t[i] = c.take<float>(n);
    r.m = c.take<float>(n);
    r.V = c.take<float>(n);
    return r;
}

// Liquid equation of state with the optional tension cut-off (section 2.5.1).
__device__ inline double pressure(const Consts &k, double rho) {
    double p = k.c2 * (rho - k.rho0);
    if (k.rho_cut > 0.0 && rho / k.rho0 < k.rho_cut) p = 0.0;
    return p;
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

struct Acc64 {
    double rs = 0.0;
    double L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double ax = 0.0, ay = 0.0, az = 0.0;
};

// One ordered pair (a target, b partner).  r = x_a - x_b, dv = v_b - v_a,
// B = T_a + T_b (six components).
__device__ inline void pair64(const Consts &k, double d2, double rx, double ry, double rz,
                              double dvx, double dvy, double dvz, double ra, double rb,
                              double Bxx, double Byy, double Bzz, double Bxy, double Bxz,
                              double Byz, double mb, double Vb, Acc64 &a) {
    const double r = sqrt(d2);
    const double q = r * k.inv_h;
    double w, f;
    if (q < 0.5) {
        w = 1.0 + q * q * (6.0 * q - 6.0);
        f = 3.0 * q - 2.0;
    } else {
        const double u = 1.0 - q;
        w = 2.0 * u * u * u;
        f = -u * u / q;
    }
    const double F = k.Fn * f;
    const double gx = F * rx, gy = F * ry, gz = F * rz;
    a.rs += mb * (k.Wn * w);
    const double tx = Vb * dvx, ty = Vb * dvy, tz = Vb * dvz;
    a.L[0] += tx * gx;
    a.L[1] += tx * gy;
    a.L[2] += tx * gz;
    a.L[3] += ty * gx;
    a.L[4] += ty * gy;
    a.L[5] += ty * gz;
    a.L[6] += tz * gx;
    a.L[7] += tz * gy;
    a.L[8] += tz * gz;
    const double wab = -(dvx * rx + dvy * ry + dvz * rz);
    double Pi = 0.0;
    if (wab < 0.0) {
        const double nu = k.h * wab / (d2 + k.epsh2);
        Pi = (-k.alpha_c * nu + k.beta * nu * nu) * 2.0 / (ra + rb);
    }
    const double bxx = Bxx - Pi, byy = Byy - Pi, bzz = Bzz - Pi;
    a.ax += mb * (bxx * gx + Bxy * gy + Bxz * gz);
    a.ay += mb * (Bxy * gx + byy * gy + Byz * gz);
    a.az += mb * (Bxz * gx + Byz * gy + bzz * gz);
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
    Kahan rs, L[9], ax, ay, az;
};

__device__ inline void pair32(const Consts32 &k, float d2, float rx, float ry, float rz, float dvx,
                              float dvy, float dvz, float ra, float rb, float Bxx, float Byy,
                              float Bzz, float Bxy, float Bxz, float Byz, float mb, float Vb,
                              Acc32 &a) {
    const float r = sqrtf(d2);
    const float q = r * k.inv_h;
    float w, f;
    if (q < 0.5f) {
        w = 1.0f + q * q * (6.0f * q - 6.0f);
        f = 3.0f * q - 2.0f;
    } else {
        const float u = 1.0f - q;
        w = 2.0f * u * u * u;
        f = -u * u / q;
    }
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
    float Pi = 0.0f;
    if (wab < 0.0f) {
        const float nu = k.h * wab / (d2 + k.epsh2);
        Pi = (-k.alpha_c * nu + k.beta * nu * nu) * 2.0f / (ra + rb);
    }
    const float bxx = Bxx - Pi, byy = Byy - Pi, bzz = Bzz - Pi;
    a.ax.add(mb * (bxx * gx + Bxy * gy + Bxz * gz));
    a.ay.add(mb * (Bxy * gx + byy * gy + Byz * gz));
    a.az.add(mb * (Bxz * gx + Byz * gy + bzz * gz));
}

// Stress rate (Hooke + Jaumann, section 2.4) and continuity for user particle a
// from its velocity gradient L (L[3 i + j] = dv_i / dx_j), written with the
// other outputs.  S~ = f_Y S;  dS = 2 mu (sym L - tr L / 3 I) + R S~ - S~ R.
__device__ inline void postpass(const Consts &k, int a, double rho, const double L[9], double ax,
                                double ay, double az, double rs, const StateDev &st,
                                const OutDev &o) {
    double S[6] = {st.sxx[a], st.syy[a], st.szz[a], st.sxy[a], st.sxz[a], st.syz[a]};
    const double f = yield_factor(k, S);
    const double sa = f * S[0], sb = f * S[1], sc = f * S[2];
    const double sd = f * S[3], se = f * S[4], sf = f * S[5];
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
    o.drho[a] = -rho * tr;
    o.ax[a] = ax;
    o.ay[a] = ay;
    o.az[a] = az;
    if (o.rho_sum) o.rho_sum[a] = rs;
}

// Cotangents of the right-hand side's outputs (user order; null = zero).
struct CotDev {
    const double *ax, *ay, *az, *drho, *ds[6], *rho_sum;
};

// Gradient destination (user order), overwritten or accumulated.
struct GradDev {
    double *x, *y, *z, *vx, *vy, *vz, *rho, *s[6];
    int accumulate;
};

// adjoint.hip
CotDev cot_dev(const sph_deriv_cot *c);
GradDev grad_dev(const sph_fields *g, int accumulate);
int check_grad(const sph_fields *g);
size_t adjoint_ws_bytes(int64_t n);
int rhs_adjoint_launch(const sph_grid *grid, const sph_state *state, const sph_params *params,
                       const CotDev &cot, const GradDev &grad, double *dparams, int accumulate_params,
                       Carve &c, hipStream_t s);
// dparams[0] (+)= sum of p0, dparams[1] (+)= sum of p1 (null parts skipped),
// fixed summation order
int reduce_params_launch(const double *p0, const double *p1, int64_t m, double *dparams,
                         int accumulate, hipStream_t s);

// host-side helpers shared by the entry points (rhs.hip)
int prepass_launch(const GridDev &g, const StateDev &st, int64_t n, const Consts &k,
                   const Rec64 &rec, int32_t *status, hipStream_t s);
int check_state(const sph_grid *grid, const sph_state *st);
int check_params(const sph_grid *grid, const sph_params *pr);
int check_deriv(const sph_deriv *o);
int rhs_launch(const sph_grid *grid, const sph_state *state, const sph_params *params,
               int precision, const sph_deriv *out, Carve &c, hipStream_t s);
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
