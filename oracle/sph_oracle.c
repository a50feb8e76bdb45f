/*
 * Plain FP64 CPU oracle for the SPH solid-body right-hand side of
 * Schaefer et al. (2016), "A smooth particle hydrodynamics code to model
 * collisions between solid, self-gravitating objects" (arXiv:1604.03290).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no source,
 * header, table or constant with the HIP library, and the HIP library never
 * calls it.
 *
 * Every quantity is evaluated as the paper writes it, in double precision,
 * one target at a time, summing over partners in ascending index order; no
 * blocking, fusion or reordering.  Build with -ffp-contract=off so that every
 * operation is rounded on its own (no fused multiply-add).
 *
 *   partners      section 3.5.2 (neighbour search): b != a, distance below h
 *   kernel        section 3.1.1 (kernel function): cubic B-spline, support h, D = 3
 *   pressure      section 2.5.1 (liquid equation of state), optional cut-off;
 *                 section 2.5.2 (Murnaghan) and 2.5.3 (Tillotson) as alternatives
 *   limiter       section 2.6 (plastic material equations), von Mises f_Y
 *   density sum   eq. (density_by_kernel_sum), section 3.1.2
 *   continuity    eq. (continuity_equation_sph), section 3.1.2
 *   momentum      eqs. (accel) and (accel_artvisc), artificial viscosity (section 3.1.3)
 *   gradient      section 3.1.6, standard SPH velocity derivative, or with the
 *                 correction tensor of the same section (linear consistency)
 *   stress rate   eqs. (stresstensor_evolution), (strain_rate_tensor), (rotation_terms),
 *                 section 2.4
 *   energy        eq. (energy_sph), section 3.1.2
 *   art. stress   section 3.1.4 (tensile instability), added to the momentum bracket
 *   XSPH          section 3.1.5, the smoothed particle velocity dx/dt
 *
 * Readings of ambiguous passages (each is also listed in the design notes):
 *   - h is the kernel's support radius, as in the kernel definition; the same
 *     h enters nu_ab (averaged smoothing length, constant h) and eps_v h^2.
 *   - the gradient in the momentum equation is taken with respect to x_a, and
 *     the artificial viscosity enters the bracket as -Pi*_ab (an additional
 *     pressure), so that pressure and viscosity both repel.
 *   - the Jaumann rotation terms are R S - S R with
 *     R = (dv^a/dx^b - dv^b/dx^a)/2, which rotates a stress carried by a
 *     rigidly spinning body with it.
 *   - f_Y = min(Y0^2 / (3 J2), 1) applied to the input S; the rotation terms
 *     use the limited stress.
 *   - mean sound speed: the linear equation of state has one sound speed c.
 *   - the density sum includes the particle's own term m_a W(0).
 *   - correction tensor: C is the inverse of the matrix of the identity the
 *     section states, M = sum_b V_b (x_b - x_a) (x) grad_a W_ab, so that M C = I
 *     (the printed definition with (x_a - x_b) contradicts that identity); the
 *     corrected gradient L C drives the strain and rotation rates, while the
 *     continuity equation keeps its own (uncorrected) sum.  Where M is singular
 *     (det M <= 1e-12 (tr M / 3)^3, e.g. fewer than three non-coplanar
 *     partners) the standard gradient is used.
 *   - energy equation: as printed, with dW/dx_b = -grad_a W; the bracket also
 *     holds -Pi*_ab I (the section on artificial viscosity adds it to the energy
 *     equation as well), i.e. the momentum bracket without artificial stress, so
 *     that sum_a m_a (v_a . dv_a/dt + du_a/dt) vanishes pair by pair.
 *   - artificial stress: a particle counts as "in tension" when its pressure is
 *     negative; then zeta_a = -eps_s sigma_a / rho_a^2 (the whole tensor), else
 *     zeta_a = 0; f = W(r_ab) / W(dmpd) with dmpd a parameter (the lattice
 *     spacing of the initial distribution), raised to the power n.
 *   - XSPH: the printed weight 2 m_b / (rho_a rho_b) is not a velocity; the
 *     weight is 2 m_b / (rho_a + rho_b) (the mean density of the pair, as in the
 *     method the section cites).
 *   - damage (section 2.7): sigma_d = -p^ I + (1 - d) f_Y S with p^ = p for p >= 0
 *     and (1 - d) p for p < 0; the damaged stress enters the momentum equation,
 *     the stress rate still evolves S.
 *   - equations of state: Murnaghan with K0 = rho0 c^2 (the liquid relation
 *     c^2 = K0 / rho0) and the same tension cut-off as the liquid equation;
 *     Tillotson with the compressed form for rho >= rho0 or u <= E_iv, the
 *     expanded form for rho < rho0 and u >= E_cv, and in between the linear
 *     interpolation in u.  The sound speed of each particle (averaged over the
 *     pair in Pi) is the thermodynamic one, c^2 = dp/drho|u + p/rho^2 dp/du|rho
 *     (floored at 0); for the liquid equation it is c.
 *
 * Layout: structure of arrays.  pos and vel are (3, n) row-major (x row, y row,
 * z row); S is (6, n) in the order xx, yy, zz, xy, xz, yz; outputs follow the
 * same layout with the target count nt in place of n; L is (9, nt) row-major
 * over (alpha, beta) with L^{alpha beta} = dv^alpha / dx^beta.
 * par = {h, rho0, c, mu, Y0, alpha, beta, eps_v, rho_cut, correction, eps_s, n_s,
 *        dmpd, xsph, eos (0 liquid, 1 Murnaghan, 2 Tillotson), n_M, a_T, b_T, A_T,
 *        B_T, E0_T, alpha_T, beta_T, E_iv, E_cv}; u (specific internal energy) is
 *        an input of the Tillotson equation (NULL = 0); dmg, the damage d in
 *        [0, 1], scales the stress (NULL = intact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { P_H, P_RHO0, P_C, P_MU, P_Y0, P_ALPHA, P_BETA, P_EPSV, P_RHOCUT, P_CORR,
       P_EPSS, P_NS, P_DMPD, P_XSPH, P_EOS, P_NM, P_AT, P_BT, P_AAT, P_BBT, P_E0T, P_ALT,
       P_BET, P_EIV, P_ECV };

/* Tillotson pressure of the compressed (cold) form, eq. (tillo1), and its partial
 * derivatives in rho and u */
static void tillotson1(const double *par, double rho, double u, double *p, double *dpr, double *dpu)
{
    const double rho0 = par[P_RHO0], a = par[P_AT], b = par[P_BT], A = par[P_AAT], B = par[P_BBT];
    const double E0 = par[P_E0T];
    const double eta = rho / rho0, chi = eta - 1.0;
    const double w = 1.0 + u / (E0 * eta * eta);
    const double dw_drho = -2.0 * u / (E0 * eta * eta * eta) / rho0;
    const double dw_du = 1.0 / (E0 * eta * eta);
    *p = (a + b / w) * rho * u + A * chi + B * chi * chi;
    *dpr = (a + b / w) * u - b / (w * w) * dw_drho * rho * u + (A + 2.0 * B * chi) / rho0;
    *dpu = (a + b / w) * rho - b / (w * w) * dw_du * rho * u;
}

/* Tillotson pressure of the expanded form, eq. (tillo2), and its partial derivatives */
static void tillotson2(const double *par, double rho, double u, double *p, double *dpr, double *dpu)
{
    const double rho0 = par[P_RHO0], a = par[P_AT], b = par[P_BT], A = par[P_AAT];
    const double E0 = par[P_E0T], al = par[P_ALT], be = par[P_BET];
    const double eta = rho / rho0, chi = eta - 1.0;
    const double w = 1.0 + u / (E0 * eta * eta);
    const double dw_drho = -2.0 * u / (E0 * eta * eta * eta) / rho0;
    const double dw_du = 1.0 / (E0 * eta * eta);
    const double z = rho0 / rho - 1.0, dz = -rho0 / (rho * rho);
    const double eb = exp(-be * z), ea = exp(-al * z * z);
    const double inner = b * rho * u / w + A * chi * eb;
    const double dinner_dr = b * u / w - b * rho * u / (w * w) * dw_drho + A / rho0 * eb
                             + A * chi * eb * (-be * dz);
    const double dinner_du = b * rho / w - b * rho * u / (w * w) * dw_du;
    *p = a * rho * u + inner * ea;
    *dpr = a * u + dinner_dr * ea + inner * ea * (-2.0 * al * z * dz);
    *dpu = a * rho + dinner_du * ea;
}

/* Pressure and squared sound speed of one particle (sections 2.5.1 to 2.5.3) */
static void eos(const double *par, double rho, double u, double *p_out, double *c2_out)
{
    const double c = par[P_C], rho0 = par[P_RHO0];
    const int kind = (int)par[P_EOS];
    double p, c2;
    if (kind == 1) { /* Murnaghan, K0 = rho0 c^2 */
        const double n = par[P_NM], K0 = rho0 * c * c, eta = rho / rho0;
        p = K0 / n * (pow(eta, n) - 1.0);
        c2 = K0 / rho0 * pow(eta, n - 1.0);
        if (par[P_RHOCUT] > 0.0 && eta < par[P_RHOCUT])
            p = 0.0;
    } else if (kind == 2) { /* Tillotson */
        double p1, r1, u1, p2, r2, u2;
        const double Eiv = par[P_EIV], Ecv = par[P_ECV];
        double dpr, dpu;
        if (rho >= rho0 || u <= Eiv) {
            tillotson1(par, rho, u, &p, &dpr, &dpu);
        } else if (u >= Ecv) {
            tillotson2(par, rho, u, &p, &dpr, &dpu);
        } else {
            tillotson1(par, rho, u, &p1, &r1, &u1);
            tillotson2(par, rho, u, &p2, &r2, &u2);
            const double t = (u - Eiv) / (Ecv - Eiv);
            p = (1.0 - t) * p1 + t * p2;
            dpr = (1.0 - t) * r1 + t * r2;
            dpu = (1.0 - t) * u1 + t * u2 + (p2 - p1) / (Ecv - Eiv);
        }
        c2 = dpr + p / (rho * rho) * dpu;
        if (c2 < 0.0)
            c2 = 0.0;
    } else { /* liquid */
        p = c * c * (rho - rho0);
        if (par[P_RHOCUT] > 0.0 && rho / rho0 < par[P_RHOCUT])
            p = 0.0;
        c2 = c * c;
    }
    *p_out = p;
    *c2_out = c2;
}

void orc_eos(int64_t n, const double *rho, const double *u, const double *par, double *p,
             double *c2)
{
    for (int64_t i = 0; i < n; ++i)
        eos(par, rho[i], u ? u[i] : 0.0, &p[i], &c2[i]);
}

static const double PI_ = 3.14159265358979323846;

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the OpenMP thread count of later calls (timing only; results do not depend on it). */
void orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* ---------------------------------------------------------------- kernel --
 * Cubic B-spline (section 3.1.1, kernel function), D = 3, s = 8/pi:
 *   W  = s/h^3 (6q^3 - 6q^2 + 1)       0 <= q < 1/2
 *      = s/h^3  2 (1 - q)^3            1/2 <= q <= 1
 *      = 0                             q > 1
 *   dW/dr = 6 s / h^4 (3q^2 - 2q)      0 <= q < 1/2
 *         = 6 s / h^4 (-(1 - q)^2)     1/2 <= q <= 1
 *         = 0                          q > 1,      q = r / h.           */
void orc_kernel(double r, double h, double *W, double *dWdr)
{
    const double s = 8.0 / PI_;
    const double q = r / h;
    const double h3 = h * h * h;
    if (q < 0.5) {
        *W = s / h3 * (6.0 * q * q * q - 6.0 * q * q + 1.0);
        *dWdr = 6.0 * s / (h3 * h) * (3.0 * q * q - 2.0 * q);
    } else if (q <= 1.0) {
        const double u = 1.0 - q;
        *W = s / h3 * 2.0 * u * u * u;
        *dWdr = 6.0 * s / (h3 * h) * (-(u * u));
    } else {
        *W = 0.0;
        *dWdr = 0.0;
    }
}

/* ------------------------------------------------------------ partners --
 * Section 3.5.2 (neighbour search): b is an interaction partner of a when b != a
 * and their distance is smaller than h.  The squared distance is formed as
 * ((dx*dx + dy*dy) + dz*dz) with dx = x_b - x_a, each operation rounded, and
 * compared strictly with h*h.                                             */
static int is_partner(const double *x, const double *y, const double *z,
                      int64_t a, int64_t b, double h2)
{
    if (a == b)
        return 0;
    const double dx = x[b] - x[a];
    const double dy = y[b] - y[a];
    const double dz = z[b] - z[a];
    const double d2 = dx * dx + dy * dy + dz * dz;
    return d2 < h2;
}

/* counts[t] = number of partners of particle targets[t] (all particles when
 * targets == NULL); returns the total.  Brute force over all n.            */
int64_t orc_count_neighbours(int64_t n, const double *pos, double h,
                             const int64_t *targets, int64_t nt, int64_t *counts)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    const double h2 = h * h;
    if (!targets)
        nt = n;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t a = targets ? targets[t] : t;
        int64_t c = 0;
        for (int64_t b = 0; b < n; ++b)
            c += is_partner(x, y, z, a, b, h2);
        counts[t] = c;
        total += c;
    }
    return total;
}

/* Partner indices of each target in ascending order into col[row_ptr[t] ..]. */
void orc_fill_neighbours(int64_t n, const double *pos, double h,
                         const int64_t *targets, int64_t nt,
                         const int64_t *row_ptr, int32_t *col)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    const double h2 = h * h;
    if (!targets)
        nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t a = targets ? targets[t] : t;
        int64_t k = row_ptr[t];
        for (int64_t b = 0; b < n; ++b)
            if (is_partner(x, y, z, a, b, h2))
                col[k++] = (int32_t)b;
    }
}

/* Indices (ascending) of all particles whose squared distance to centre is
 * below radius^2.  Returns the count; writes at most cap indices.          */
int64_t orc_ball(int64_t n, const double *pos, const double *centre, double radius,
                 int64_t *out, int64_t cap)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    const double r2 = radius * radius;
    int64_t k = 0;
    for (int64_t b = 0; b < n; ++b) {
        const double dx = x[b] - centre[0];
        const double dy = y[b] - centre[1];
        const double dz = z[b] - centre[2];
        if (dx * dx + dy * dy + dz * dz < r2) {
            if (k < cap)
                out[k] = b;
            ++k;
        }
    }
    return k;
}

/* ------------------------------------------------------------- prepass --
 * Per particle:
 *   p      = c^2 (rho - rho0), set to 0 when rho_cut > 0 and rho/rho0 < rho_cut
 *            (section 2.5.1, liquid equation of state and its tension cut-off)
 *   J2     = S^{ab} S^{ab} / 2 over all nine entries (section 2.6)
 *   f_Y    = min(Y0^2 / (3 J2), 1)                 (section 2.6)
 *   sigma  = -p delta + f_Y S                      (section 2.2)
 * Outputs p (n), fy (n), sigma (6, n).                                     */
static void to_matrix(const double *s6, int64_t n, int64_t i, double M[3][3])
{
    M[0][0] = s6[0 * n + i];
    M[1][1] = s6[1 * n + i];
    M[2][2] = s6[2 * n + i];
    M[0][1] = M[1][0] = s6[3 * n + i];
    M[0][2] = M[2][0] = s6[4 * n + i];
    M[1][2] = M[2][1] = s6[5 * n + i];
}

static void one_prepass(int64_t n, int64_t i, const double *rho, const double *u,
                        const double *dmg, const double *S, const double *par, double *p_out,
                        double *f_out, double *cs_out, double sig[3][3])
{
    const double Y0 = par[P_Y0];
    double p, c2;
    eos(par, rho[i], u ? u[i] : 0.0, &p, &c2);
    *cs_out = sqrt(c2);
    double Sm[3][3];
    to_matrix(S, n, i, Sm);
    double J2 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            J2 += Sm[a][b] * Sm[a][b];
    J2 *= 0.5;
    double f = 1.0;
    if (3.0 * J2 > Y0 * Y0)
        f = Y0 * Y0 / (3.0 * J2);
    const double d = dmg ? dmg[i] : 0.0;
    const double ph = p >= 0.0 ? p : (1.0 - d) * p; /* damage relieves tension only */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            sig[a][b] = (1.0 - d) * f * Sm[a][b] - (a == b ? ph : 0.0);
    *p_out = p;
    *f_out = f;
}

void orc_prepass(int64_t n, const double *rho, const double *S, const double *par,
                 double *p, double *fy, double *sigma)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double sig[3][3], cs;
        one_prepass(n, i, rho, NULL, NULL, S, par, &p[i], &fy[i], &cs, sig);
        sigma[0 * n + i] = sig[0][0];
        sigma[1 * n + i] = sig[1][1];
        sigma[2 * n + i] = sig[2][2];
        sigma[3 * n + i] = sig[0][1];
        sigma[4 * n + i] = sig[0][2];
        sigma[5 * n + i] = sig[1][2];
    }
}

/* prepass with the specific internal energy and the damage (NULL = 0) */
void orc_prepass2(int64_t n, const double *rho, const double *u, const double *dmg,
                  const double *S, const double *par, double *p, double *fy, double *cs,
                  double *sigma)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double sig[3][3];
        one_prepass(n, i, rho, u, dmg, S, par, &p[i], &fy[i], &cs[i], sig);
        sigma[0 * n + i] = sig[0][0];
        sigma[1 * n + i] = sig[1][1];
        sigma[2 * n + i] = sig[2][2];
        sigma[3 * n + i] = sig[0][1];
        sigma[4 * n + i] = sig[0][2];
        sigma[5 * n + i] = sig[1][2];
    }
}

/* ----------------------------------------------------------------- RHS --
 * For each target a = targets[t] (t = 0..nt-1; all particles when targets is
 * NULL) over its partners b = col[row_ptr[t] .. row_ptr[t+1]) in the given
 * (ascending) order.  With r_ab = x_a - x_b, r = |r_ab| and
 * grad_a W_ab = (dW/dr)(r) r_ab / r (zero when r = 0):
 *
 *   rho_sum_a = m_a W(0) + sum_b m_b W_ab                      (density sum)
 *   drho_a    = rho_a sum_b (m_b/rho_b) (v_a - v_b) . grad_a W_ab   (continuity)
 *   L_a^{ab}  = sum_b (m_b/rho_b) (v_b - v_a)^alpha d W_ab / d x_a^beta
 *   w_ab      = (v_a - v_b) . (x_a - x_b)
 *   nu_ab     = h w_ab / (|r_ab|^2 + eps_v h^2)
 *   Pi*_ab    = (-alpha c nu_ab + beta nu_ab^2) / ((rho_a + rho_b)/2) if w_ab < 0, else 0
 *   a_a^alpha = sum_b m_b [sigma_a/rho_a^2 + sigma_b/rho_b^2 - Pi*_ab I]^{alpha beta}
 *                    d W_ab / d x_a^beta
 *   edot = (L + L^T)/2,  R = (L - L^T)/2,  S~ = f_Y S
 *   dS_a = 2 mu (edot - tr(edot) I / 3) + R S~ - S~ R
 *
 * With the correction, L is replaced by L C before the stress rate.
 *
 * Outputs (per target): acc (3, nt), drho (nt), dS (6, nt), rho_sum (nt),
 * and L (9, nt) when L != NULL: the gradient that drives the stress rate
 * (L C with the correction).                                               */
/* C = M^{-1} by the adjugate when M is regular (see the reading in the header),
 * the identity otherwise.  Returns 1 when the inverse was taken. */
static int correction_tensor(const double M[3][3], double C[3][3])
{
    double A[3][3];
    A[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    A[0][1] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
    A[0][2] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
    A[1][0] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    A[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
    A[1][2] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
    A[2][0] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    A[2][1] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
    A[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    const double det = M[0][0] * A[0][0] + M[0][1] * A[1][0] + M[0][2] * A[2][0];
    const double t = (M[0][0] + M[1][1] + M[2][2]) / 3.0;
    if (!(det > 1e-12 * t * t * t) || !isfinite(det)) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                C[i][j] = i == j ? 1.0 : 0.0;
        return 0;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[i][j] = A[i][j] / det;
    return 1;
}

/* du (nullable): specific internal energy rate; xv (nullable, (3, nt)): dx/dt */
void orc_rhs2(int64_t n, const double *pos, const double *vel, const double *rho,
              const double *u, const double *dmg, const double *S, const double *m,
              const double *par,
              const int64_t *targets, int64_t nt, const int64_t *row_ptr, const int32_t *col,
              double *acc, double *drho, double *dS, double *rho_sum, double *Lout,
              double *du, double *xv)
{
    const double h = par[P_H], mu = par[P_MU];
    const double alpha = par[P_ALPHA], beta = par[P_BETA], eps_v = par[P_EPSV];
    const int corr = par[P_CORR] != 0.0;
    const double eps_s = par[P_EPSS], n_s = par[P_NS], xsph = par[P_XSPH];
    double Wmpd = 1.0, dWmpd;
    if (eps_s > 0.0)
        orc_kernel(par[P_DMPD], h, &Wmpd, &dWmpd);
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    const double *vx = vel, *vy = vel + n, *vz = vel + 2 * n;
    if (!targets)
        nt = n;

    /* per-particle stress (prepass) for every particle */
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *fy = (double *)malloc(sizeof(double) * (size_t)n);
    double *cs = (double *)malloc(sizeof(double) * (size_t)n);
    double *sg = (double *)malloc(sizeof(double) * 6 * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double sig[3][3];
        one_prepass(n, i, rho, u, dmg, S, par, &p[i], &fy[i], &cs[i], sig);
        sg[0 * n + i] = sig[0][0];
        sg[1 * n + i] = sig[1][1];
        sg[2 * n + i] = sig[2][2];
        sg[3 * n + i] = sig[0][1];
        sg[4 * n + i] = sig[0][2];
        sg[5 * n + i] = sig[1][2];
    }

    double W0, dW0;
    orc_kernel(0.0, h, &W0, &dW0);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t a = targets ? targets[t] : t;
        const double xa[3] = {x[a], y[a], z[a]};
        const double va[3] = {vx[a], vy[a], vz[a]};
        const double ra = rho[a];
        double siga[3][3];
        to_matrix(sg, n, a, siga);

        double rs = m[a] * W0;
        double cont = 0.0;
        double ac[3] = {0.0, 0.0, 0.0};
        double ue = 0.0;                    /* energy sum */
        double xs[3] = {0.0, 0.0, 0.0};     /* XSPH sum */
        const int tens_a = p[a] < 0.0;
        double L[3][3] = {{0.0}};
        double Mc[3][3] = {{0.0}}; /* sum_b V_b (x_b - x_a) (x) grad_a W_ab */

        for (int64_t k = row_ptr[t]; k < row_ptr[t + 1]; ++k) {
            const int64_t b = col[k];
            const double xb[3] = {x[b], y[b], z[b]};
            const double vb[3] = {vx[b], vy[b], vz[b]};
            const double rb = rho[b];
            double sigb[3][3];
            to_matrix(sg, n, b, sigb);

            double rv[3], r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                rv[d] = xa[d] - xb[d];
                r2 += rv[d] * rv[d];
            }
            const double r = sqrt(r2);
            double W, dW;
            orc_kernel(r, h, &W, &dW);
            double gW[3] = {0.0, 0.0, 0.0};
            if (r > 0.0)
                for (int d = 0; d < 3; ++d)
                    gW[d] = dW * rv[d] / r;

            /* density sum */
            rs += m[b] * W;

            /* continuity and velocity gradient */
            const double Vb = m[b] / rb;
            for (int al = 0; al < 3; ++al)
                cont += Vb * (va[al] - vb[al]) * gW[al];
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be)
                    L[al][be] += Vb * (vb[al] - va[al]) * gW[be];
            if (corr)
                for (int al = 0; al < 3; ++al)
                    for (int ga = 0; ga < 3; ++ga)
                        Mc[al][ga] += Vb * (xb[al] - xa[al]) * gW[ga];

            /* artificial viscosity */
            double wab = 0.0;
            for (int d = 0; d < 3; ++d)
                wab += (va[d] - vb[d]) * rv[d];
            double Pi = 0.0;
            if (wab < 0.0) {
                const double nu = h * wab / (r2 + eps_v * h * h);
                const double cbar = 0.5 * (cs[a] + cs[b]);
                Pi = (-alpha * cbar * nu + beta * nu * nu) / (0.5 * (ra + rb));
            }

            /* artificial stress factor (zeta_a + zeta_b) f^n, zeta = -eps_s sigma / rho^2 in tension */
            const int tens_b = p[b] < 0.0;
            double fn = 0.0;
            if (eps_s > 0.0 && (tens_a || tens_b))
                fn = pow(W / Wmpd, n_s);

            /* momentum (with artificial stress) and energy (without it) */
            for (int al = 0; al < 3; ++al) {
                double s = 0.0;
                for (int be = 0; be < 3; ++be) {
                    const double B = siga[al][be] / (ra * ra) + sigb[al][be] / (rb * rb)
                                     - (al == be ? Pi : 0.0);
                    double zeta = 0.0;
                    if (tens_a)
                        zeta += -eps_s * siga[al][be] / (ra * ra);
                    if (tens_b)
                        zeta += -eps_s * sigb[al][be] / (rb * rb);
                    s += (B + zeta * fn) * gW[be];
                    /* energy: (1/2) m_b B (v_a - v_b)^al dW/dx_b^be, dW/dx_b = -gW */
                    ue += 0.5 * m[b] * B * (va[al] - vb[al]) * (-gW[be]);
                }
                ac[al] += m[b] * s;
            }

            /* XSPH: 2 m_b / (rho_a + rho_b) (v_b - v_a) W */
            for (int d = 0; d < 3; ++d)
                xs[d] += 2.0 * m[b] / (ra + rb) * (vb[d] - va[d]) * W;
        }

        /* corrected velocity gradient L C (the continuity sum above stays as printed) */
        if (corr) {
            double C[3][3], Lc[3][3];
            correction_tensor(Mc, C);
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be) {
                    double v = 0.0;
                    for (int ga = 0; ga < 3; ++ga)
                        v += L[al][ga] * C[ga][be];
                    Lc[al][be] = v;
                }
            memcpy(L, Lc, sizeof L);
        }

        /* stress rate: Hooke term plus Jaumann rotation terms on the limited S */
        double St[3][3];
        to_matrix(S, n, a, St);
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be)
                St[al][be] *= fy[a];
        double ed[3][3], R[3][3];
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) {
                ed[al][be] = 0.5 * (L[al][be] + L[be][al]);
                R[al][be] = 0.5 * (L[al][be] - L[be][al]);
            }
        const double tr = ed[0][0] + ed[1][1] + ed[2][2];
        double dSm[3][3];
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) {
                double rot = 0.0;
                for (int g = 0; g < 3; ++g)
                    rot += R[al][g] * St[g][be] - St[al][g] * R[g][be];
                dSm[al][be] = 2.0 * mu * (ed[al][be] - (al == be ? tr / 3.0 : 0.0)) + rot;
            }

        for (int d = 0; d < 3; ++d)
            acc[d * nt + t] = ac[d];
        drho[t] = ra * cont;
        dS[0 * nt + t] = dSm[0][0];
        dS[1 * nt + t] = dSm[1][1];
        dS[2 * nt + t] = dSm[2][2];
        dS[3 * nt + t] = dSm[0][1];
        dS[4 * nt + t] = dSm[0][2];
        dS[5 * nt + t] = dSm[1][2];
        rho_sum[t] = rs;
        if (du)
            du[t] = ue;
        if (xv)
            for (int d = 0; d < 3; ++d)
                xv[d * nt + t] = va[d] + xsph * xs[d];
        if (Lout)
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be)
                    Lout[(al * 3 + be) * nt + t] = L[al][be];
    }
    free(p);
    free(fy);
    free(cs);
    free(sg);
}

void orc_rhs(int64_t n, const double *pos, const double *vel, const double *rho,
             const double *S, const double *m, const double *par,
             const int64_t *targets, int64_t nt, const int64_t *row_ptr, const int32_t *col,
             double *acc, double *drho, double *dS, double *rho_sum, double *Lout)
{
    orc_rhs2(n, pos, vel, rho, NULL, NULL, S, m, par, targets, nt, row_ptr, col, acc, drho, dS,
             rho_sum, Lout, NULL, NULL);
}
