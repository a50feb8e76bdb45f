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
#include "common.hpp"
#include "rhs_common.hpp"
#include "timing.hpp"

namespace sph {
namespace {

// --------------------------------------------------------------- prepass --
__global__ __launch_bounds__(kBlock) void k_prepass(GridDev g, StateDev st, int64_t n, Consts k,
                                                    Rec64 rec, int32_t *__restrict__ status) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = g.perm[s];
    const double x = st.x[a], y = st.y[a], z = st.z[a];
    if (!within_cell(g, (int)s, x, y, z)) raise_flag(status, SPH_ERR_STALE_GRID);
    const double rho = st.rho[a];
    if (!(rho > 0.0) || !isfinite(rho)) raise_flag(status, SPH_ERR_DOMAIN);
    double S[6] = {st.sxx[a], st.syy[a], st.szz[a], st.sxy[a], st.sxz[a], st.syz[a]};
    const double p = pressure(k, rho);
    const double f = yield_factor(k, S);
    const double ir2 = 1.0 / (rho * rho);
    rec.x[s] = x;
    rec.y[s] = y;
    rec.z[s] = z;
    rec.vx[s] = st.vx[a];
    rec.vy[s] = st.vy[a];
    rec.vz[s] = st.vz[a];
    rec.rho[s] = rho;
    rec.t[0][s] = (f * S[0] - p) * ir2;
    rec.t[1][s] = (f * S[1] - p) * ir2;
    rec.t[2][s] = (f * S[2] - p) * ir2;
    rec.t[3][s] = f * S[3] * ir2;
    rec.t[4][s] = f * S[4] * ir2;
    rec.t[5][s] = f * S[5] * ir2;
    const double m = st.m[a];
    rec.m[s] = m;
    rec.V[s] = m / rho;
}

// FP32 copies of the pair operands (positions stay FP64 for the exact test)
__global__ __launch_bounds__(kBlock) void k_narrow(Rec64 rec, int64_t n, Rec32 r32) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    r32.vx[s] = (float)rec.vx[s];
    r32.vy[s] = (float)rec.vy[s];
    r32.vz[s] = (float)rec.vz[s];
    r32.rho[s] = (float)rec.rho[s];
#pragma unroll
    for (int c = 0; c < 6; ++c) r32.t[c][s] = (float)rec.t[c][s];
    r32.m[s] = (float)rec.m[s];
    r32.V[s] = (float)rec.V[s];
}

// ---------------------------------------------------------- pairs, FP64 --
__global__ __launch_bounds__(kBlock) void k_pairs64(GridDev g, int64_t n, Consts k, Rec64 rec,
                                                    StateDev st, OutDev out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double xa = rec.x[s], ya = rec.y[s], za = rec.z[s];
    const double vxa = rec.vx[s], vya = rec.vy[s], vza = rec.vz[s];
    const double ra = rec.rho[s];
    const double ta0 = rec.t[0][s], ta1 = rec.t[1][s], ta2 = rec.t[2][s];
    const double ta3 = rec.t[3][s], ta4 = rec.t[4][s], ta5 = rec.t[5][s];
    Acc64 acc;
    acc.rs = rec.m[s] * k.Wn;  // own term m_a W(0)
    for_each_row(g, xa, ya, za, k.reach, [&](int s0, int s1) {
        for (int t = s0; t < s1; ++t) {
            const double xb = rec.x[t], yb = rec.y[t], zb = rec.z[t];
            const double d2 = dist2_exact(xa, ya, za, xb, yb, zb);
            if (!(d2 < k.h2) || t == s) continue;
            pair64(k, d2, xa - xb, ya - yb, za - zb, rec.vx[t] - vxa, rec.vy[t] - vya,
                   rec.vz[t] - vza, ra, rec.rho[t], ta0 + rec.t[0][t], ta1 + rec.t[1][t],
                   ta2 + rec.t[2][t], ta3 + rec.t[3][t], ta4 + rec.t[4][t], ta5 + rec.t[5][t],
                   rec.m[t], rec.V[t], acc);
        }
    });
    postpass(k, g.perm[s], ra, acc.L, acc.ax, acc.ay, acc.az, acc.rs, st, out);
}

// ----------------------------------------- pairs, FP32 + Kahan sums --
__global__ __launch_bounds__(kBlock) void k_pairs32(GridDev g, int64_t n, Consts k, Rec64 rec,
                                                    Rec32 r32, StateDev st, OutDev out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double xa = rec.x[s], ya = rec.y[s], za = rec.z[s];
    const float vxa = r32.vx[s], vya = r32.vy[s], vza = r32.vz[s];
    const float ra = r32.rho[s];
    const float ta0 = r32.t[0][s], ta1 = r32.t[1][s], ta2 = r32.t[2][s];
    const float ta3 = r32.t[3][s], ta4 = r32.t[4][s], ta5 = r32.t[5][s];
    const Consts32 kf = narrow(k);
    Acc32 acc;
    for_each_row(g, xa, ya, za, k.reach, [&](int s0, int s1) {
        for (int t = s0; t < s1; ++t) {
            const double xb = rec.x[t], yb = rec.y[t], zb = rec.z[t];
            const double d2 = dist2_exact(xa, ya, za, xb, yb, zb);
            if (!(d2 < k.h2) || t == s) continue;
            pair32(kf, (float)d2, (float)(xa - xb), (float)(ya - yb), (float)(za - zb),
                   r32.vx[t] - vxa, r32.vy[t] - vya, r32.vz[t] - vza, ra, r32.rho[t],
                   ta0 + r32.t[0][t], ta1 + r32.t[1][t], ta2 + r32.t[2][t], ta3 + r32.t[3][t],
                   ta4 + r32.t[4][t], ta5 + r32.t[5][t], r32.m[t], r32.V[t], acc);
        }
    });
    double L[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) L[c] = acc.L[c].value();
    const double rs = rec.m[s] * k.Wn + acc.rs.value();
    postpass(k, g.perm[s], rec.rho[s], L, acc.ax.value(), acc.ay.value(), acc.az.value(), rs, st,
             out);
}

}  // namespace

int prepass_launch(const GridDev &g, const StateDev &st, int64_t n, const Consts &k,
                   const Rec64 &rec, int32_t *status, hipStream_t s) {
    k_prepass<<<blocks_for(n), kBlock, 0, s>>>(g, st, n, k, rec, status);
    SPH_LAUNCHED();
    return SPH_OK;
}

size_t rhs_ws_bytes(int64_t n) {
    Carve c(nullptr);
    carve_rec64(c, n);
    carve_rec32(c, n);
    return c.used;
}

int check_state(const sph_grid *grid, const sph_state *st) {
    if (!st) return fail(SPH_ERR_INVALID_ARG, "state is NULL");
    if (st->n != grid->n) return fail(SPH_ERR_INVALID_ARG, "state n differs from grid n");
    const double *p[] = {st->x,   st->y,   st->z,   st->vx,  st->vy,  st->vz,  st->rho,
                         st->sxx, st->syy, st->szz, st->sxy, st->sxz, st->syz, st->m};
    for (const double *q : p)
        if (!q) return fail(SPH_ERR_INVALID_ARG, "state array is NULL");
    return SPH_OK;
}

int check_params(const sph_grid *grid, const sph_params *pr) {
    if (!pr) return fail(SPH_ERR_INVALID_ARG, "params is NULL");
    const double v[] = {pr->h,     pr->rho0, pr->c,     pr->mu,     pr->Y0,
                        pr->alpha, pr->beta, pr->eps_v, pr->rho_cut};
    for (double q : v)
        if (!std::isfinite(q)) return fail(SPH_ERR_INVALID_ARG, "non-finite parameter");
    if (!(pr->h > 0.0) || !(pr->rho0 > 0.0) || !(pr->c > 0.0))
        return fail(SPH_ERR_INVALID_ARG, "h, rho0 and c must be positive");
    if (pr->mu < 0.0 || !(pr->Y0 > 0.0) || pr->eps_v <= 0.0 || pr->rho_cut < 0.0)
        return fail(SPH_ERR_INVALID_ARG, "mu >= 0, Y0 > 0, eps_v > 0, rho_cut >= 0 required");
    if (pr->h > grid->h) return fail(SPH_ERR_INVALID_ARG, "h exceeds the grid's support radius");
    return SPH_OK;
}

int check_deriv(const sph_deriv *o) {
    if (!o) return fail(SPH_ERR_INVALID_ARG, "output is NULL");
    const double *p[] = {o->ax, o->ay, o->az, o->drho, o->dsxx, o->dsyy, o->dszz,
                         o->dsxy, o->dsxz, o->dsyz};
    for (const double *q : p)
        if (!q) return fail(SPH_ERR_INVALID_ARG, "output array is NULL");
    return SPH_OK;
}

// Forward right-hand side on a carved workspace (also used by the leapfrog).
int rhs_launch(const sph_grid *grid, const sph_state *state, const sph_params *params,
               int precision, const sph_deriv *out, Carve &c, hipStream_t s) {
    const int64_t n = grid->n;
    GridDev g = grid_dev(grid);
    Consts k = make_consts(*params, g.delta);
    Rec64 rec = carve_rec64(c, n);
    Rec32 r32 = carve_rec32(c, n);
    StateDev st = state_dev(state);
    OutDev od = out_dev(out);
    int rc = prepass_launch(g, st, n, k, rec, c.status(), s);
    if (rc) return rc;
    if (precision == SPH_FP64) {
        TimedRegion t("pairs_fp64", s);
        k_pairs64<<<blocks_for(n), kBlock, 0, s>>>(g, n, k, rec, st, od);
        SPH_LAUNCHED();
    } else {
        k_narrow<<<blocks_for(n), kBlock, 0, s>>>(rec, n, r32);
        SPH_LAUNCHED();
        TimedRegion t("pairs_fp32comp", s);
        k_pairs32<<<blocks_for(n), kBlock, 0, s>>>(g, n, k, rec, r32, st, od);
        SPH_LAUNCHED();
    }
    return SPH_OK;
}

}  // namespace sph

using namespace sph;

extern "C" int sph_rhs(const sph_grid *grid, const sph_state *state, const sph_params *params,
                       int precision, const sph_deriv *out, void *ws, size_t ws_bytes,
                       void *stream) {
    clear_error();
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_state(grid, state)) ||
        (rc = check_params(grid, params)) || (rc = check_deriv(out)))
        return rc;
    if (precision != SPH_FP64 && precision != SPH_FP32_COMP)
        return fail(SPH_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (!ws) return fail(SPH_ERR_INVALID_ARG, "workspace is NULL");
    const size_t need = rhs_ws_bytes(grid->n);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = clear_status(ws, s))) return rc;
    Carve c(ws);
    return rhs_launch(grid, state, params, precision, out, c, s);
}
