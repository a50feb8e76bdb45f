// Kick-drift-kick leapfrog on a frozen grid and its reverse sweep.
//
//   F_0 = F(x_0, U_0),  U = (v, rho, S)
//   for n = 0 .. K-1:
//     U'      = U_n + dt/2 F_n,   S' <- f_Y(S') S'         (kick)
//     x_{n+1} = x_n + dt v'                               (drift)
//     F_{n+1} = F(x_{n+1}, U')
//     U_{n+1} = U' + dt/2 F_{n+1}, S <- f_Y(S) S          (kick)
//
// f_Y = min(Y0^2 / (3 J2), 1) is the von Mises factor of section 2.6.  The
// trajectory is integrated in the grid's slot order (the state is permuted once
// at the start and back at the end), so every per-particle pass reads and
// writes contiguous arrays.  The checkpoint of step k holds (x_k, v_k, rho_k,
// S_k, F_k), the velocity gradient behind F_k and, with the correction tensor,
// its moment matrix: 38 arrays of n doubles in slot order.  The reverse sweep walks the steps backwards, recomputing U' from
// the checkpoint, and applies in turn the adjoints of the second kick, of the
// right-hand side at (x_{n+1}, U'), of the drift and of the first kick.
#include "adjoint.hpp"
#include "common.hpp"
#include "rhs_common.hpp"

namespace sph {
namespace {

constexpr int kArrays = 38;  // x3 v3 rho S6 | a3 drho dS6 | L and M (slot order, vgrad_width values per slot)
constexpr int kLOffset = 23;

struct Fields13 {
    double *p[13];  // x y z vx vy vz rho sxx syy szz sxy sxz syz
};

struct Deriv10 {
    double *p[10];  // ax ay az drho dsxx .. dsyz
};

__device__ inline void limit6(double S[6], double Y0sq) {
    const double j3 = 3.0 * j2_of(S);
    if (j3 > Y0sq) {
        const double f = Y0sq / j3;
#pragma unroll
        for (int i = 0; i < 6; ++i) S[i] *= f;
    }
}

// The kick at one particle: v += h a, rho += h drho, S = f_Y(S + h dS)(S + h dS).
// Every kick of the forward pass and its recomputation in the reverse sweep go
// through this one function, so they round identically.
__device__ inline void kick_at(double v[3], double &rho, double S[6], const double F[10], double h,
                               double Y0sq) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = v[c] + h * F[c];
    rho = rho + h * F[3];
#pragma unroll
    for (int c = 0; c < 6; ++c) S[c] = S[c] + h * F[4 + c];
    limit6(S, Y0sq);
}

// One pass between two right-hand sides: with kick2 the second kick of the
// previous step (U_k = kick(U', F_k)); with slab the checkpoint (U_k, F_k); with
// kick1 the first kick and the drift of the next step (U' = kick(U_k, F_k),
// x += dt v') and the operand records of the next right-hand side (its prepass).
__global__ __launch_bounds__(kBlock) void k_advance(Fields13 u, Deriv10 d, double *slab, int64_t n,
                                                    double h, double dt, double Y0sq, int kick2,
                                                    int kick1, GridDev g, Consts k,
                                                    const double *__restrict__ m,
                                                    double *__restrict__ rec,
                                                    int32_t *__restrict__ status,
                                                    const double *__restrict__ dmg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[3], rho, S[6], F[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) F[c] = d.p[c][i];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = u.p[3 + c][i];
    rho = u.p[6][i];
#pragma unroll
    for (int c = 0; c < 6; ++c) S[c] = u.p[7 + c][i];
    if (kick2) kick_at(v, rho, S, F, h, Y0sq);
    if (slab) {
#pragma unroll
        for (int c = 0; c < 3; ++c) slab[c * n + i] = u.p[c][i];
#pragma unroll
        for (int c = 0; c < 3; ++c) slab[(3 + c) * n + i] = v[c];
        slab[6 * n + i] = rho;
#pragma unroll
        for (int c = 0; c < 6; ++c) slab[(7 + c) * n + i] = S[c];
#pragma unroll
        for (int c = 0; c < 10; ++c) slab[(13 + c) * n + i] = F[c];
    }
    if (kick1) {
        kick_at(v, rho, S, F, h, Y0sq);
        double x[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c] = u.p[c][i] + dt * v[c];
            u.p[c][i] = x[c];
        }
        write_rec(g, k, i, x[0], x[1], x[2], v[0], v[1], v[2], rho, S, m[i], rec, status, 0.0,
                  dmg ? dmg[i] : 0.0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) u.p[3 + c][i] = v[c];
    u.p[6][i] = rho;
#pragma unroll
    for (int c = 0; c < 6; ++c) u.p[7 + c][i] = S[c];
}

// user order -> slot order: dst[c][s] = src[c][perm[s]] (a null source gives 0)
struct Src14 {
    const double *p[14];
};
struct Dst14 {
    double *p[14];
};

__global__ __launch_bounds__(kBlock) void k_to_slots(Src14 src, Dst14 dst, int nc,
                                                     const int32_t *__restrict__ perm, int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = perm[s];
    for (int c = 0; c < nc; ++c) dst.p[c][s] = src.p[c] ? src.p[c][a] : 0.0;
}

// slot order -> user order: dst[c][perm[s]] = src[c][s]
__global__ __launch_bounds__(kBlock) void k_to_users(Src14 src, Dst14 dst, int nc,
                                                     const int32_t *__restrict__ perm, int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int a = perm[s];
    for (int c = 0; c < nc; ++c) dst.p[c][a] = src.p[c][s];
}

__global__ __launch_bounds__(kBlock) void k_fill(double *p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Adjoint of the kick U_out = kick(U_in, F) at particle i: given S_in, dS and
// the cotangent of U_out in gU (updated in place to the cotangent of U_in),
// writes or adds the cotangent of F into gF (and, with Fout, returns its new
// value there); returns the Y0 contribution.
__device__ inline double kick_adj_at(const double S_in[6], const double dS[6], const Fields13 &gU,
                                     const Deriv10 &gF, int64_t i, double h, double Y0,
                                     int accumulate, double *Fout = nullptr) {
    double S[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) S[c] = S_in[c] + h * dS[c];
    double Sb[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) Sb[c] = gU.p[7 + c][i];
    const double j2 = j2_of(S);
    const double Y0sq = Y0 * Y0;
    double out[6], y0p = 0.0;
    if (3.0 * j2 > Y0sq) {
        const double f = Y0sq / (3.0 * j2);
        double fb = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) fb += Sb[c] * S[c];
        const double Jb = -fb * f / j2;
#pragma unroll
        for (int c = 0; c < 6; ++c) out[c] = f * Sb[c] + Jb * (c < 3 ? S[c] : 2.0 * S[c]);
        y0p = fb * 2.0 * f / Y0;
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) out[c] = Sb[c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) gU.p[7 + c][i] = out[c];
    double v[10];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = h * gU.p[3 + c][i];
    v[3] = h * gU.p[6][i];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[4 + c] = h * out[c];
#pragma unroll
    for (int c = 0; c < 10; ++c) {
        const double r = accumulate ? gF.p[c][i] + v[c] : v[c];
        gF.p[c][i] = r;
        if (Fout) Fout[c] = r;
    }
    return y0p;
}

// Reverse sweep, first pass of step k: recompute U' = kick(U_k, F_k) into Up
// and apply the adjoint of the second kick U_{k+1} = kick(U', F_{k+1}); then the
// first stages of the adjoint of F_{k+1} = F(x_{k+1}, U'): its operand records
// (prepass) and its post stage, from the checkpointed velocity gradient L_{k+1}
// and the cotangent of F_{k+1} just completed.  The Y0 and mu contributions are
// added to the block's accumulators.
__global__ __launch_bounds__(kBlock) void k_rev_kick2(Fields13 Uk, Deriv10 Fk, Fields13 Up,
                                                      Deriv10 Fk1, Fields13 gU, Deriv10 gF,
                                                      int64_t n, double h, double Y0,
                                                      int accumulate, double *acc_y0,
                                                      const double *__restrict__ x1,
                                                      const double *__restrict__ L1, GridDev g,
                                                      Consts k, const double *__restrict__ m,
                                                      double *__restrict__ rec, AdjRec ad,
                                                      double *acc_mu, int32_t *__restrict__ status,
                                                      const double *__restrict__ dmg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double y0p = 0.0, mup = 0.0;
    if (i < n) {
        double v[3], rho = Uk.p[6][i], S[6], F[10], dS[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = Uk.p[3 + c][i];
#pragma unroll
        for (int c = 0; c < 6; ++c) S[c] = Uk.p[7 + c][i];
#pragma unroll
        for (int c = 0; c < 10; ++c) F[c] = Fk.p[c][i];
        kick_at(v, rho, S, F, h, Y0 * Y0);
#pragma unroll
        for (int c = 0; c < 3; ++c) Up.p[3 + c][i] = v[c];
        Up.p[6][i] = rho;
#pragma unroll
        for (int c = 0; c < 6; ++c) Up.p[7 + c][i] = S[c];
#pragma unroll
        for (int c = 0; c < 6; ++c) dS[c] = Fk1.p[4 + c][i];
        double cF[10];
        y0p = kick_adj_at(S, dS, gU, gF, i, h, Y0, accumulate, cF);
        const double mi = m[i];
        write_rec(g, k, i, x1[i], x1[n + i], x1[2 * n + i], v[0], v[1], v[2], rho, S, mi, rec,
                  status, 0.0, dmg ? dmg[i] : 0.0);
        double L[9];
        const double *Li = L1 + (size_t)i * vgrad_width(k.corr);
#pragma unroll
        for (int c = 0; c < 9; ++c) L[c] = Li[c];
        double M[6] = {0, 0, 0, 0, 0, 0};
        if (k.corr) {
#pragma unroll
            for (int c = 0; c < 6; ++c) M[c] = Li[9 + c];
        }
        const double c6[6] = {cF[4], cF[5], cF[6], cF[7], cF[8], cF[9]};
        mup = adj_post_at(k, i, L, k.corr, M, rho, S, c6, cF[3], cF[0], cF[1], cF[2], 0.0, ad);
    }
    const double tot = block_sum(y0p);
    const double tot_mu = block_sum(mup);
    if (threadIdx.x == 0) {
        acc_y0[blockIdx.x] += tot;
        acc_mu[blockIdx.x] += tot_mu;
    }
}

// Reverse sweep, last pass of step k: adjoint of the drift (vbar += dt xbar),
// then of the first kick U' = kick(U_k, F_k) (fresh cotangent of F_k).
__global__ __launch_bounds__(kBlock) void k_rev_kick1(Fields13 Uk, Deriv10 Fk, Fields13 gU,
                                                      Deriv10 gF, int64_t n, double h, double dt,
                                                      double Y0, double *acc_y0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double y0p = 0.0;
    if (i < n) {
#pragma unroll
        for (int c = 0; c < 3; ++c) gU.p[3 + c][i] += dt * gU.p[c][i];
        double S[6], dS[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            S[c] = Uk.p[7 + c][i];
            dS[c] = Fk.p[4 + c][i];
        }
        y0p = kick_adj_at(S, dS, gU, gF, i, h, Y0, 0);
    }
    const double tot = block_sum(y0p);
    if (threadIdx.x == 0) acc_y0[blockIdx.x] += tot;
}

Fields13 fields_of(const sph_fields *f) {
    return Fields13{{f->x, f->y, f->z, f->vx, f->vy, f->vz, f->rho, f->sxx, f->syy, f->szz, f->sxy,
                     f->sxz, f->syz}};
}

Fields13 slab_fields(double *slab, int64_t n) {
    Fields13 f;
    for (int c = 0; c < 13; ++c) f.p[c] = slab + c * n;
    return f;
}

Deriv10 slab_deriv(double *slab, int64_t n) {
    Deriv10 d;
    for (int c = 0; c < 10; ++c) d.p[c] = slab + (13 + c) * n;
    return d;
}

Deriv10 carve_deriv(Carve &c, int64_t n) {
    Deriv10 d;
    for (int i = 0; i < 10; ++i) d.p[i] = c.take<double>(n);
    return d;
}

Fields13 carve_fields(Carve &c, int64_t n) {
    Fields13 f;
    for (int i = 0; i < 13; ++i) f.p[i] = c.take<double>(n);
    return f;
}

sph_deriv deriv_struct(const Deriv10 &d) {
    sph_deriv o;
    o.ax = d.p[0];
    o.ay = d.p[1];
    o.az = d.p[2];
    o.drho = d.p[3];
    o.dsxx = d.p[4];
    o.dsyy = d.p[5];
    o.dszz = d.p[6];
    o.dsxy = d.p[7];
    o.dsxz = d.p[8];
    o.dsyz = d.p[9];
    o.rho_sum = nullptr;
    o.du = o.dx = o.dy = o.dz = nullptr;
    o.dd3 = nullptr;
    o.n_act = nullptr;
    o.vgrad = nullptr;  // the leapfrog hands the velocity gradient over itself
    o.rec = nullptr;    // and keeps its records in its workspace
    return o;
}

sph_state state_struct(const Fields13 &f, const double *m, int64_t n, const double *d) {
    sph_state s;
    s.n = n;
    s.x = f.p[0];
    s.y = f.p[1];
    s.z = f.p[2];
    s.vx = f.p[3];
    s.vy = f.p[4];
    s.vz = f.p[5];
    s.rho = f.p[6];
    s.sxx = f.p[7];
    s.syy = f.p[8];
    s.szz = f.p[9];
    s.sxy = f.p[10];
    s.sxz = f.p[11];
    s.syz = f.p[12];
    s.m = m;
    s.u = nullptr;
    s.d = d;
    s.flaw_ptr = nullptr;
    s.flaw_eps = nullptr;
    return s;
}

// state (13 arrays) and masses, user order -> slot order
int state_to_slots(const sph_grid *grid, const sph_state *src, const Fields13 &dst, double *m,
                   hipStream_t s) {
    const Src14 a{{src->x, src->y, src->z, src->vx, src->vy, src->vz, src->rho, src->sxx,
                   src->syy, src->szz, src->sxy, src->sxz, src->syz, src->m}};
    Dst14 b;
    for (int c = 0; c < 13; ++c) b.p[c] = dst.p[c];
    b.p[13] = m;
    k_to_slots<<<blocks_for(grid->n), kBlock, 0, s>>>(a, b, 14, grid->perm, grid->n);
    SPH_LAUNCHED();
    return SPH_OK;
}

// damage, user order -> slot order (held fixed over the trajectory)
int damage_to_slots(const sph_grid *grid, const double *d, double *dst, hipStream_t s) {
    Src14 a;
    Dst14 b;
    for (int c = 0; c < 14; ++c) {
        a.p[c] = nullptr;
        b.p[c] = nullptr;
    }
    a.p[0] = d;
    b.p[0] = dst;
    k_to_slots<<<blocks_for(grid->n), kBlock, 0, s>>>(a, b, 1, grid->perm, grid->n);
    SPH_LAUNCHED();
    return SPH_OK;
}

// 13 fields, slot order -> user order
int fields_to_users(const sph_grid *grid, const Fields13 &src, const Fields13 &dst, hipStream_t s) {
    Src14 a;
    Dst14 b;
    for (int c = 0; c < 13; ++c) {
        a.p[c] = src.p[c];
        b.p[c] = dst.p[c];
    }
    a.p[13] = nullptr;
    b.p[13] = nullptr;
    k_to_users<<<blocks_for(grid->n), kBlock, 0, s>>>(a, b, 13, grid->perm, grid->n);
    SPH_LAUNCHED();
    return SPH_OK;
}

GradDev grad_of(const Fields13 &f) {
    return GradDev{f.p[0], f.p[1], f.p[2], f.p[3], f.p[4], f.p[5], f.p[6],
                   {f.p[7], f.p[8], f.p[9], f.p[10], f.p[11], f.p[12]}, 1};
}

int check_lf(const sph_grid *grid, const sph_state *s0, const sph_params *params, double dt,
             int steps) {
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_state(grid, s0)) || (rc = check_params(grid, params)))
        return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SPH_ERR_INVALID_ARG, "dt must be positive");
    if (steps < 1) return fail(SPH_ERR_INVALID_ARG, "steps must be >= 1");
    if (params->xsph != 0.0)
        return fail(SPH_ERR_NOT_IMPLEMENTED, "the leapfrog drifts with v (no XSPH)");
    if (params->eos == 2.0)
        return fail(SPH_ERR_NOT_IMPLEMENTED, "the leapfrog does not evolve u (Tillotson)");
    return SPH_OK;
}

}  // namespace

size_t leapfrog_ws_bytes(int64_t n) {
    Carve c(nullptr);
    carve_deriv(c, n);   // F, slot order
    carve_fields(c, n);  // state, slot order
    c.take<double>(n);   // masses, slot order
    c.take<double>(n);   // damage, slot order
    c.used += rhs_ws_bytes(n);
    return c.used;
}

size_t leapfrog_adjoint_ws_bytes(int64_t n) {
    Carve c(nullptr);
    carve_fields(c, n);  // cotangent of the state, slot order
    carve_fields(c, n);  // U' (only v, rho, S used; x points at the next checkpoint)
    carve_deriv(c, n);   // cotangent of F_{n+1}
    carve_deriv(c, n);   // cotangent of F_n
    c.take<double>(n);   // masses, slot order
    c.take<double>(n);   // damage, slot order
    c.take<double>(blocks_for(n) + blocks_for(n, 64));  // mu and Y0 accumulators
    c.used += adjoint_ws_bytes(n);
    return c.used;
}

}  // namespace sph

using namespace sph;

extern "C" size_t sph_checkpoint_bytes(int64_t n, int steps) {
    if (n <= 0 || steps < 0) return 0;
    return (size_t)(steps + 1) * kArrays * (size_t)n * sizeof(double);
}

extern "C" int sph_leapfrog(const sph_grid *grid, const sph_state *s0, const sph_params *params,
                            double dt, int steps, const sph_fields *s_final, double *checkpoints,
                            void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_lf(grid, s0, params, dt, steps)) || (rc = check_grad(s_final))) return rc;
    if (!ws) return fail(SPH_ERR_INVALID_ARG, "workspace is NULL");
    const int64_t n = grid->n;
    const size_t need = leapfrog_ws_bytes(n);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = clear_status(ws, s))) return rc;
    Carve c(ws);
    Deriv10 F = carve_deriv(c, n);
    const Fields13 U = carve_fields(c, n);
    double *m = c.take<double>(n);
    double *dmg = c.take<double>(n);
    Carve rc_ws(ws);  // the right-hand side shares the status word, carves after these
    rc_ws.used = c.used;
    if ((rc = state_to_slots(grid, s0, U, m, s))) return rc;
    if (s0->d && (rc = damage_to_slots(grid, s0->d, dmg, s))) return rc;
    if (!s0->d) dmg = nullptr;
    const sph_state st = state_struct(U, m, n, dmg);
    const sph_deriv d = deriv_struct(F);
    const double half = 0.5 * dt;
    const unsigned nb = blocks_for(n);
    auto rhs = [&](int k) {
        Carve w = rc_ws;
        double *Lout = checkpoints ? checkpoints + ((size_t)k * kArrays + kLOffset) * n : nullptr;
        return rhs_launch(grid, &st, params, SPH_FP64, &d, w, s, Lout, true, k > 0);
    };
    const double Y0sq = params->Y0 * params->Y0;
    auto slab = [&](int k) { return checkpoints ? checkpoints + (size_t)k * kArrays * n : nullptr; };
    GridDev g = grid_dev(grid);
    g.io = nullptr;
    const Consts kc = make_consts(*params, g.delta);
    double *rec = rhs_rec_of(rc_ws, n);
    int32_t *status = c.status();
    if ((rc = rhs(0))) return rc;
    for (int k = 0; k < steps; ++k) {
        k_advance<<<nb, kBlock, 0, s>>>(U, F, slab(k), n, half, dt, Y0sq, k > 0, 1, g, kc, m, rec,
                                        status, dmg);
        SPH_LAUNCHED();
        if ((rc = rhs(k + 1))) return rc;
    }
    k_advance<<<nb, kBlock, 0, s>>>(U, F, slab(steps), n, half, dt, Y0sq, 1, 0, g, kc, m, rec,
                                    status, dmg);
    SPH_LAUNCHED();
    return fields_to_users(grid, U, fields_of(s_final), s);
}

extern "C" int sph_leapfrog_adjoint(const sph_grid *grid, const sph_state *s0,
                                    const sph_params *params, double dt, int steps,
                                    const double *checkpoints, const sph_cfields *cot_final,
                                    const sph_fields *grad0, double *dparams, void *ws,
                                    size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_lf(grid, s0, params, dt, steps)) || (rc = check_grad(grad0))) return rc;
    if (!checkpoints || !cot_final || !dparams || !ws)
        return fail(SPH_ERR_INVALID_ARG, "null pointer");
    const int64_t n = grid->n;
    const size_t need = leapfrog_adjoint_ws_bytes(n);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = clear_status(ws, s))) return rc;
    Carve c(ws);
    const Fields13 gU = carve_fields(c, n);  // cotangent of the current state, slot order
    Fields13 Up = carve_fields(c, n);
    Deriv10 gF1 = carve_deriv(c, n);
    Deriv10 gF0 = carve_deriv(c, n);
    double *m = c.take<double>(n);
    double *dmg = c.take<double>(n);
    // mu accumulators per block, then Y0 per block (kicks) or per wavefront (pairs)
    const unsigned nw = blocks_for(n, 64);
    double *parts = c.take<double>(blocks_for(n) + nw);
    Carve adj_ws(ws);
    adj_ws.used = c.used;
    const unsigned nb = blocks_for(n);
    const double half = 0.5 * dt;
    double *ck = const_cast<double *>(checkpoints);
    const double Y0 = params->Y0;

    // cotangent of the final state and the masses, into slot order
    {
        const Src14 a{{cot_final->x, cot_final->y, cot_final->z, cot_final->vx, cot_final->vy,
                       cot_final->vz, cot_final->rho, cot_final->sxx, cot_final->syy,
                       cot_final->szz, cot_final->sxy, cot_final->sxz, cot_final->syz, s0->m}};
        Dst14 b;
        for (int i = 0; i < 13; ++i) b.p[i] = gU.p[i];
        b.p[13] = m;
        k_to_slots<<<nb, kBlock, 0, s>>>(a, b, 14, grid->perm, n);
        SPH_LAUNCHED();
    }
    if (s0->d && (rc = damage_to_slots(grid, s0->d, dmg, s))) return rc;
    if (!s0->d) dmg = nullptr;
    k_fill<<<blocks_for(nb + nw), kBlock, 0, s>>>(parts, nb + nw, 0.0);
    SPH_LAUNCHED();
    double *acc_y0 = parts + nb;

    const GradDev acc = grad_of(gU);
    auto adjoint_at = [&](const sph_state &st, const Deriv10 &gF, const double *slab,
                          bool post_ready) {
        CotDev cot{gF.p[0], gF.p[1], gF.p[2], gF.p[3],
                   {gF.p[4], gF.p[5], gF.p[6], gF.p[7], gF.p[8], gF.p[9]}, nullptr};
        Carve w = adj_ws;
        return rhs_adjoint_launch(grid, &st, params, cot, acc, dparams, 1, w, s,
                                  slab + (size_t)kLOffset * n, true, parts, post_ready);
    };
    // buffers of the fused prepass and post stage (those of rhs_adjoint_launch)
    GridDev g = grid_dev(grid);
    g.io = nullptr;
    const Consts kc = make_consts(*params, g.delta);
    Carve ab_ws = adj_ws;
    const AdjBuffers ab = adj_buffers(ab_ws, n);
    int32_t *status = c.status();

    for (int k = steps - 1; k >= 0; --k) {
        double *slab_k = ck + (size_t)k * kArrays * n;
        double *slab_k1 = ck + (size_t)(k + 1) * kArrays * n;
        const Fields13 Uk = slab_fields(slab_k, n);
        const Deriv10 Fk = slab_deriv(slab_k, n);
        const Fields13 Uk1 = slab_fields(slab_k1, n);
        const Deriv10 Fk1 = slab_deriv(slab_k1, n);
        // U' = kick(U_k, F_k) (its positions are x_{k+1}), then the adjoint of the
        // second kick U_{k+1} = kick(U', F_{k+1}): cotangent of U' and of F_{k+1}
        // (F_{k+1} already holds the first kick of step k+1 unless k+1 = steps)
        k_rev_kick2<<<nb, kBlock, 0, s>>>(Uk, Fk, Up, Fk1, gU, gF1, n, half, Y0,
                                          k + 1 < steps ? 1 : 0, acc_y0, Uk1.p[0],
                                          slab_k1 + (size_t)kLOffset * n, g, kc, m, ab.rec,
                                          ab.ad, parts, status, dmg);
        SPH_LAUNCHED();
        Fields13 Upx = Up;
        for (int c3 = 0; c3 < 3; ++c3) Upx.p[c3] = Uk1.p[c3];
        // right-hand side F_{k+1} = F(x_{k+1}, U'): its pair stage
        const sph_state st1 = state_struct(Upx, m, n, dmg);
        if ((rc = adjoint_at(st1, gF1, slab_k1, true))) return rc;
        // drift x_{k+1} = x_k + dt v', then the first kick U' = kick(U_k, F_k):
        // cotangent of U_k, fresh cotangent of F_k
        k_rev_kick1<<<nb, kBlock, 0, s>>>(Uk, Fk, gU, gF0, n, half, dt, Y0, acc_y0);
        SPH_LAUNCHED();
        Deriv10 tmp = gF1;
        gF1 = gF0;
        gF0 = tmp;
    }
    // F_0 = F(x_0, U_0)
    const sph_state st0 = state_struct(slab_fields(ck, n), m, n, dmg);
    if ((rc = adjoint_at(st0, gF1, ck, false))) return rc;
    // dparams = the accumulators summed in a fixed order
    if ((rc = reduce_params_launch(parts, nb, acc_y0, nw, dparams, 0, s))) return rc;
    return fields_to_users(grid, gU, fields_of(grad0), s);
}
