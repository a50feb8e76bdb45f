// Vector-Jacobian product of the right-hand side (double precision).
//
// Forward quantities are recomputed from the state: the prepass records
// (T = sigma / rho^2, V = m / rho, slot order) and every particle's velocity
// gradient L.  Then, in the reverse order of the forward passes:
//
//  post     per particle a, from the cotangents of drho = -rho tr L and
//           dS = 2 mu dev(sym L) + R S~ - S~ R (section 2.4), with G the
//           symmetric matrix of the dS cotangent (off-diagonal = half the stored
//           component's cotangent):
//             Lbar = -rho drho_bar I + 2 mu dev(G) + (G S~ - S~ G)
//             mu_bar += 2 <dev G, L>,  rho_bar += -tr(L) drho_bar,
//             S~_bar += G R - R G
//  pairs    gather form: particle c loops over its partners b once and takes
//           the derivative of every term it appears in, as target (sums of c)
//           and as partner (sums of b).  With r = x_c - x_b, u = v_b - v_c,
//           g = grad_c W_cb = F(r) r, A = m_b abar_c - m_c abar_b and
//           M = V_b Lbar_c + V_c Lbar_b:
//             gbar  = M^T u + (T_c + T_b - Pi I) A,   Pibar = -A . g
//             xbar_c += (rsbar_c m_b + rsbar_b m_c) g + F gbar + G (r.gbar) r
//                       - wbar u + 2 r2bar r
//             vbar_c += -M g + wbar r
//             Tbar_c += sym(A (x) g),  Vbar_c += u^T Lbar_b g,
//             rhobar_c += -Pibar Pi / (rho_c + rho_b)
//           where G = F'(r)/r and wbar, r2bar follow from Pibar through
//           nu = h w / (r^2 + eps h^2), w = (v_c - v_b).r (approaching pairs).
//           No atomics: every particle writes only its own gradient.
//  pre      per particle: through T = (f_Y S - p I)/rho^2, V = m/rho, the
//           pressure (section 2.5.1) and the limiter f_Y = min(Y0^2/(3 J2), 1)
//           (section 2.6) to rho_bar, S_bar and Y0_bar.  With the Murnaghan
//           equation (section 2.5.2) dp/drho = K0/rho0 eta^(n-1) and Pi's mean
//           sound speed (c_c + c_b)/2 carries rho too: cbar_c += Pibar dPi/dcbar / 2
//           per pair, rho_bar += cbar_c c_c (n - 1) / (2 rho_c).  With Tillotson
//           (section 2.5.3) c^2 = D = p_rho + p p_u / rho^2, whose partials D_rho and
//           D_u come from evaluating the region's form on first-order jets in (rho, u):
//           rho_bar += cbar_c D_rho / (2 c), u_bar += cbar_c D_u / (2 c) + p^_u tr(Tbar)
//           (-1/rho^2), the partner's sound speed and tension read from its record's
//           signed c.  The artificial stress
//           (section 3.1.4) adds Z = (zeta_c + zeta_b) f^n to B, zeta = -eps_s T in
//           tension (p < 0, for the liquid and Murnaghan equations rho < rho0 outside
//           the cut-off), f = w(q)/w(dmpd):
//           Tbar_c gains the factor 1 + zeta_c/T_c f^n and
//           xbar_c += (A . (zeta_c + zeta_b) g) n f^(n-1) g / (w(dmpd) Wn).  The
//           cotangents ubar of du/dt and chi of dx/dt (sections 3.1.2, 3.1.5) add,
//           with e = (m_b ubar_c + m_c ubar_b)/2, Be = T_c + T_b - Pi I and
//           kappa = m_b chi_c - m_c chi_b:
//             gbar += e Be u, vbar_c -= e Be g, Tbar_c += e sym(u (x) g),
//             Pibar -= e u.g (energy), and vbar_c -= xsph 2 W kappa / S,
//             xbar_c += xsph 2 (kappa.u) g / S, rhobar_c -= xsph 2 W (kappa.u) / S^2
//             with S = rho_c + rho_b (XSPH); vbar_c += chi_c (dx/dt = v + ...).  With a damage field d
//           (section 2.7, held fixed) T = ((1 - d) f_Y S - p^ I)/rho^2: the
//           deviator's cotangent carries the factor 1 - d, and so does the
//           pressure's slope where p < 0.
//
// mu_bar and Y0_bar are reduced per block with a fixed tree and then by one
// block in a fixed order, so results are reproducible bit for bit.
#include <type_traits>

#include "adjoint.hpp"
#include "common.hpp"
#include "rhs_common.hpp"
#include "timing.hpp"

namespace sph {

namespace {

__device__ inline double ld(const double *p, int i) { return p ? p[i] : 0.0; }

__device__ inline void put(double *p, int i, double v, int acc) {
    if (acc)
        p[i] += v;
    else
        p[i] = v;
}

// moment matrix of the correction (xx yy zz xy xz yz) += P r r^T, P = -V F
__device__ inline void moment_add(double M[6], double V, double F, double rx, double ry, double rz) {
    const double P = -V * F;
    const double px = P * rx, py = P * ry, pz = P * rz;
    M[0] = fma(px, rx, M[0]);
    M[1] = fma(py, ry, M[1]);
    M[2] = fma(pz, rz, M[2]);
    M[3] = fma(px, ry, M[3]);
    M[4] = fma(px, rz, M[4]);
    M[5] = fma(py, rz, M[5]);
}

// forward velocity gradient (and with the correction its moment matrix) of every slot
template <bool kCorr>
__global__ __launch_bounds__(kBlock) void k_adj_L(GridDev g, int64_t n, Consts k,
                                                  const double *__restrict__ rec, AdjRec ad) {
    const int64_t s = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (s >= n) return;
    const double2 *ra = rec2(rec, s);
    const double2 p0 = ra[0], p1 = ra[1], p2 = ra[2];
    const double xa = p0.x, ya = p0.y, za = p1.x, vxa = p1.y, vya = p2.x, vza = p2.y;
    double L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double M[6] = {0, 0, 0, 0, 0, 0};
    for_each_candidate(g, s, xa, ya, za, k.reach, [&](int t) {
        const double2 *rb = rec2(rec, t);
        const double2 b0 = rb[0], b1 = rb[1];
        const double d2 = dist2_exact(xa, ya, za, b0.x, b0.y, b1.x);
        if (!(d2 < k.h2)) return;
        const double2 b2 = rb[2], b3 = rb[3];
        const KernelPieces kp = kernel_pieces(k, d2, rsqrt64(d2));
        const double F = k.Fn * kp.f;
        const double gx = F * (xa - b0.x), gy = F * (ya - b0.y), gz = F * (za - b1.x);
        const double V = b3.y;
        const double tx = V * (b1.y - vxa), ty = V * (b2.x - vya), tz = V * (b2.y - vza);
        L[0] = fma(tx, gx, L[0]); L[1] = fma(tx, gy, L[1]); L[2] = fma(tx, gz, L[2]);
        L[3] = fma(ty, gx, L[3]); L[4] = fma(ty, gy, L[4]); L[5] = fma(ty, gz, L[5]);
        L[6] = fma(tz, gx, L[6]); L[7] = fma(tz, gy, L[7]); L[8] = fma(tz, gz, L[8]);
        if (kCorr) moment_add(M, V, F, xa - b0.x, ya - b0.y, za - b1.x);
    });
    store_vgrad<kCorr>(ad.L, s, L, M);
}

// same over the frozen pair list with cooperative gathers of the partners' first
// four chunks (position, velocity, density, V: 64 bytes), kSplit wavefronts per block
// of 64 slots as in the forward list kernels
template <bool kCorr>
__global__ __launch_bounds__(64 * kSplit) void k_adj_L_list(GridDev g, int64_t n, Consts k,
                                                            const double *__restrict__ rec,
                                                            AdjRec ad) {
    __shared__ double2 lbuf[kSplit][64 * 4];
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
    double2 p0 = make_double2(0, 0), p1 = p0, p2 = p0;
    if (act) {
        const double2 *ra = rec2(rec, s);
        p0 = ra[0]; p1 = ra[1]; p2 = ra[2];
    }
    const double xa = p0.x, ya = p0.y, za = p1.x, vxa = p1.y, vya = p2.x, vza = p2.y;
    double v[kCorr ? 15 : 9];
#pragma unroll
    for (int i = 0; i < (kCorr ? 15 : 9); ++i) v[i] = 0.0;
    double *L = v, *M = v + 9;  // M: the moment matrix (kCorr)
    const char *recs = reinterpret_cast<const char *>(rec);
    const int32_t *row = g.pl_slot + base + __lane_id();
    // one step ahead, as in the pair kernels
    if (q < steps) gather_dma4(recs, kRec * 8, row[(int64_t)q << 6], buf);
    int nxt = q + kSplit < steps ? row[(int64_t)(q + kSplit) << 6] : 0;
    for (int j = q; j < steps; j += kSplit) {
        wait_vm();
        const double2 b0 = dma4_chunk(buf, 0), b1 = dma4_chunk(buf, 1), b2 = dma4_chunk(buf, 2),
                      b3 = dma4_chunk(buf, 3);
        wave_sync();
        if (j + kSplit < steps) {
            gather_dma4(recs, kRec * 8, nxt, buf);
            if (j + 2 * kSplit < steps) nxt = row[(int64_t)(j + 2 * kSplit) << 6];
        }
        if (j < cnt) {
            const double d2 = dist2_exact(xa, ya, za, b0.x, b0.y, b1.x);
            if (d2 < k.h2) {
                const KernelPieces kp = kernel_pieces(k, d2, rsqrt64(d2));
                const double F = k.Fn * kp.f;
                const double gx = F * (xa - b0.x), gy = F * (ya - b0.y), gz = F * (za - b1.x);
                const double V = b3.y;
                const double tx = V * (b1.y - vxa), ty = V * (b2.x - vya), tz = V * (b2.y - vza);
                L[0] = fma(tx, gx, L[0]); L[1] = fma(tx, gy, L[1]); L[2] = fma(tx, gz, L[2]);
                L[3] = fma(ty, gx, L[3]); L[4] = fma(ty, gy, L[4]); L[5] = fma(ty, gz, L[5]);
                L[6] = fma(tz, gx, L[6]); L[7] = fma(tz, gy, L[7]); L[8] = fma(tz, gz, L[8]);
                if (kCorr) moment_add(M, V, F, xa - b0.x, ya - b0.y, za - b1.x);
            }
        }
    }
    fold_waves<kSplit, kSplit * 64 * 4 * 2>(v, reinterpret_cast<double *>(lbuf));
    if (q != 0 || !act) return;
    store_vgrad<kCorr>(ad.L, s, L, M);
}

// post stage (see the file header); with inv (user-order state and cotangents, the
// inverse permutation) thread i takes user particle i, reading those arrays in order
__global__ __launch_bounds__(kBlock) void k_adj_post(GridDev g, int64_t n, Consts k,
                                                     const double *__restrict__ rec, StateDev st,
                                                     CotDev cot, AdjRec ad,
                                                     const int32_t *__restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mu_part = 0.0;
    if (i < n) {
        const int64_t s = inv ? (int64_t)inv[i] : i;
        const int a = inv ? (int)i : io_index(g, s);
        double L[9], c6[6];
        const double *Ls = ad.L + (size_t)s * ad.lw;
#pragma unroll
        for (int i = 0; i < 9; ++i) L[i] = Ls[i];
        const double S[6] = {st.sxx[a], st.syy[a], st.szz[a], st.sxy[a], st.sxz[a], st.syz[a]};
#pragma unroll
        for (int i = 0; i < 6; ++i) c6[i] = ld(cot.ds[i], a);
        double M[6] = {0, 0, 0, 0, 0, 0};
        if (k.corr) {
#pragma unroll
            for (int i = 0; i < 6; ++i) M[i] = Ls[9 + i];
        }
        mu_part = adj_post_at(k, s, L, k.corr, M, rec[s * kRec + 6], S, c6,
                              ld(cot.drho, a), ld(cot.ax, a), ld(cot.ay, a), ld(cot.az, a),
                              ld(cot.rho_sum, a), ad);
        if (cot.du || cot.dx[0] || cot.dx[1] || cot.dx[2]) {
            ad.ext[0][s] = ld(cot.du, a);
#pragma unroll
            for (int i = 0; i < 3; ++i) ad.ext[1 + i][s] = ld(cot.dx[i], a);
        }
    }
    const double tot = block_sum(mu_part);
    if (threadIdx.x == 0) put(ad.part_mu, blockIdx.x, tot, ad.add_parts);
}

struct AdjAcc {
    double gx = 0, gy = 0, gz = 0, gvx = 0, gvy = 0, gvz = 0, grho = 0, gV = 0;
    double gT[6] = {0, 0, 0, 0, 0, 0};
    double gc = 0;  // cotangent of the particle's sound speed (Murnaghan)
};

// The sums of the P wavefronts of the list kernel's workgroup added into wavefront 0
// (fold_waves, in wavefront order).
template <int P, int Cap>
__device__ inline void fold_adj(AdjAcc &a, double *scratch) {
    double v[15] = {a.gx, a.gy, a.gz, a.gvx, a.gvy, a.gvz, a.grho, a.gV,
                    a.gT[0], a.gT[1], a.gT[2], a.gT[3], a.gT[4], a.gT[5], a.gc};
    fold_waves<P, Cap>(v, scratch);
    a.gx = v[0]; a.gy = v[1]; a.gz = v[2]; a.gvx = v[3]; a.gvy = v[4]; a.gvz = v[5];
    a.grho = v[6]; a.gV = v[7];
#pragma unroll
    for (int i = 0; i < 6; ++i) a.gT[i] = v[8 + i];
    a.gc = v[14];
}

// Own data of particle c in the pair stage.
struct AdjOwn {
    double xc, yc, zc, vxc, vyc, vzc, rc, mc, Vc, Tc[6], Lbc[9], abx, aby, abz, rsc;
    double cc;  // sound speed (the forward record's, sign bit cleared)
    bool tens;  // negative pressure (the record's sign bit)
};

// Murnaghan sound speed of a partner from its density, as the forward prepass forms it
__device__ inline double murnaghan_c(const Consts &k, double rho) {
    const double eta = rho / k.rho0;
    const double en1 = pow(eta, k.n_M - 1.0);
    return sqrt(k.K0 / k.rho0 * en1);
}

// Both roles of the pair (c, b) (see the file header).  b = forward record chunks
// b0..b6 of the partner (its mass is V rho), e0..e6 = its adjoint record chunks.  With the
// correction, Mc and Mb are the symmetrised cotangents of the moment matrices
// of c and b, whose terms P r r^T (P = -V_b F, r = x_c - x_b) add
//   xbar_c += -[V_b (2 F Mc r + (r.Mc r) G r) + V_c (2 F Mb r + (r.Mb r) G r)],
//   Vbar_c += -F (r.Mb r).
template <bool kCorr = false, int kEos = 0, bool kAS = false, bool kXC = false>
__device__ inline void adj_pair(const Consts &k, const AdjOwn &o, double d2, double2 b0,
                                double2 b1, double2 b2, double2 b3, double2 b4, double2 b5,
                                double2 b6, double2 e0, double2 e1, double2 e2, double2 e3,
                                double2 e4, double2 e5, double2 e6, AdjAcc &acc,
                                const double *Mc = nullptr, const double *Mb = nullptr,
                                const double *xo = nullptr, const double *xb = nullptr,
                                double cb = 0.0 /* Tillotson: partner's signed c */) {
    const double Gn = k.Fn * k.inv_h * k.inv_h;
    const double Lbb[9] = {e0.x, e0.y, e1.x, e1.y, e2.x, e2.y, e3.x, e3.y, e4.x};
    const double rx = o.xc - b0.x, ry = o.yc - b0.y, rz = o.zc - b1.x;
    const double ux = b1.y - o.vxc, uy = b2.x - o.vyc, uz = b2.y - o.vzc;
    const double rb_ = b3.x, Vb = b3.y, mb = Vb * rb_;
    const double ir = rsqrt64(d2);
    const KernelPieces kp = kernel_pieces(k, d2, ir);
    // G = F'(r) / r:  3 Gn / q inside, Gn (1 - q^2) / q^3 outside (0 at r = 0)
    const double iq = k.h * ir;
    const double Gi = 3.0 * Gn * iq;
    const double Go = Gn * (1.0 - kp.q * kp.q) * iq * iq * iq;
    const double G = d2 > 0.0 ? (kp.inner ? Gi : Go) : 0.0;
    const double F = k.Fn * kp.f;
    const double gx = F * rx, gy = F * ry, gz = F * rz;
    const double Ax = mb * o.abx - o.mc * e4.y;
    const double Ay = mb * o.aby - o.mc * e5.x;
    const double Az = mb * o.abz - o.mc * e5.y;
    double M[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) M[i] = Vb * o.Lbc[i] + o.Vc * Lbb[i];
    const double w = -(ux * rx + uy * ry + uz * rz);
    double alpha_c = k.alpha_c;
    if constexpr (kEos == 1) alpha_c = k.alpha * (0.5 * (o.cc + murnaghan_c(k, rb_)));
    if constexpr (kEos == 2) alpha_c = k.alpha * (0.5 * (o.cc + fabs(cb)));
    const Visc vs = viscosity(k, d2, w, o.rc, rb_, alpha_c);
    const double Pi = vs.Pi;
    double B0 = o.Tc[0] + b4.x - Pi, B1 = o.Tc[1] + b4.y - Pi;
    double B2 = o.Tc[2] + b5.x - Pi, B3 = o.Tc[3] + b5.y;
    double B4 = o.Tc[4] + b6.x, B5 = o.Tc[5] + b6.y;
    const double Be[6] = {B0, B1, B2, B3, B4, B5};  // the energy bracket (no artificial stress)
    // artificial stress: Z0 = zeta_c + zeta_b, fn = f^n, dfn = n f^(n-1) / (w(dmpd) Wn)
    double Z0[6] = {0, 0, 0, 0, 0, 0}, fn = 0.0, dfn = 0.0, zc = 0.0;
    if constexpr (kAS) {
        const bool tb = kEos == 2 ? signbit(cb)
                                  : rb_ < k.rho0 && !(k.rho_cut > 0.0 && rb_ / k.rho0 < k.rho_cut);
        if (o.tens || tb) {
            const double f = kp.w * k.inv_wm;
            if (k.n_int > 0) {
                fn = f;
                for (int e = 1; e < k.n_int; ++e) fn *= f;
            } else {
                fn = pow_frac(f, k.n_s);
            }
            dfn = f > 0.0 ? k.n_s * (fn / f) * k.inv_wm / k.Wn : 0.0;
            zc = o.tens ? -k.eps_s : 0.0;
            const double zb = tb ? -k.eps_s : 0.0;
            const double Tb[6] = {b4.x, b4.y, b5.x, b5.y, b6.x, b6.y};
#pragma unroll
            for (int i = 0; i < 6; ++i) Z0[i] = zc * o.Tc[i] + zb * Tb[i];
            B0 += Z0[0] * fn; B1 += Z0[1] * fn; B2 += Z0[2] * fn;
            B3 += Z0[3] * fn; B4 += Z0[4] * fn; B5 += Z0[5] * fn;
        }
    }
    double gbx = M[0] * ux + M[3] * uy + M[6] * uz + B0 * Ax + B3 * Ay + B4 * Az;
    double gby = M[1] * ux + M[4] * uy + M[7] * uz + B3 * Ax + B1 * Ay + B5 * Az;
    double gbz = M[2] * ux + M[5] * uy + M[8] * uz + B4 * Ax + B5 * Ay + B2 * Az;
    double Pib = -(Ax * gx + Ay * gy + Az * gz);
    double rxs = 0.0;  // XSPH: xbar_c += rxs g
    if constexpr (kXC) {
        const double e = 0.5 * (mb * xo[0] + o.mc * xb[0]);
        gbx += e * (Be[0] * ux + Be[3] * uy + Be[4] * uz);
        gby += e * (Be[3] * ux + Be[1] * uy + Be[5] * uz);
        gbz += e * (Be[4] * ux + Be[5] * uy + Be[2] * uz);
        acc.gvx -= e * (Be[0] * gx + Be[3] * gy + Be[4] * gz);
        acc.gvy -= e * (Be[3] * gx + Be[1] * gy + Be[5] * gz);
        acc.gvz -= e * (Be[4] * gx + Be[5] * gy + Be[2] * gz);
        acc.gT[0] += e * (ux * gx);
        acc.gT[1] += e * (uy * gy);
        acc.gT[2] += e * (uz * gz);
        acc.gT[3] += e * (ux * gy + uy * gx);
        acc.gT[4] += e * (ux * gz + uz * gx);
        acc.gT[5] += e * (uy * gz + uz * gy);
        Pib -= e * (ux * gx + uy * gy + uz * gz);
        const double kx = mb * xo[1] - o.mc * xb[1], ky = mb * xo[2] - o.mc * xb[2],
                     kz = mb * xo[3] - o.mc * xb[3];
        const double iS = 1.0 / (o.rc + rb_);
        const double e2 = 2.0 * k.xsph * iS, Wv = k.Wn * kp.w;
        const double ku = kx * ux + ky * uy + kz * uz;
        acc.gvx -= e2 * Wv * kx;
        acc.gvy -= e2 * Wv * ky;
        acc.gvz -= e2 * Wv * kz;
        rxs = e2 * ku;
        acc.grho -= e2 * Wv * iS * ku;
    }
    double wb = 0.0, r2b = 0.0;
    if (w < 0.0) {
        const double nub = Pib * (-alpha_c + 2.0 * k.beta * vs.nu) * vs.coef;
        wb = nub * k.h * vs.invD;
        r2b = -nub * vs.nu * vs.invD;
        acc.grho -= Pib * Pi * 0.5 * vs.coef;  // Pi / (rho_c + rho_b)
        if constexpr (kEos) acc.gc += Pib * (-k.alpha * vs.nu * vs.coef) * 0.5;
    }
    double rsw = o.rsc * mb + e6.x * o.mc + rxs;
    if constexpr (kAS) {
        // d(f^n)/dx_c = dfn g: the scalar A . (Z0 g) rides on the g direction
        const double zx = Z0[0] * gx + Z0[3] * gy + Z0[4] * gz;
        const double zy = Z0[3] * gx + Z0[1] * gy + Z0[5] * gz;
        const double zz = Z0[4] * gx + Z0[5] * gy + Z0[2] * gz;
        rsw += (Ax * zx + Ay * zy + Az * zz) * dfn;
    }
    const double rg = rx * gbx + ry * gby + rz * gbz;
    acc.gx += rsw * gx + F * gbx + G * rg * rx - wb * ux + 2.0 * r2b * rx;
    acc.gy += rsw * gy + F * gby + G * rg * ry - wb * uy + 2.0 * r2b * ry;
    acc.gz += rsw * gz + F * gbz + G * rg * rz - wb * uz + 2.0 * r2b * rz;
    acc.gvx += -(M[0] * gx + M[1] * gy + M[2] * gz) + wb * rx;
    acc.gvy += -(M[3] * gx + M[4] * gy + M[5] * gz) + wb * ry;
    acc.gvz += -(M[6] * gx + M[7] * gy + M[8] * gz) + wb * rz;
    const double tf = kAS ? 1.0 + zc * fn : 1.0;  // d(T_c + zeta_c f^n)/dT_c
    acc.gT[0] += (Ax * gx) * tf;
    acc.gT[1] += (Ay * gy) * tf;
    acc.gT[2] += (Az * gz) * tf;
    acc.gT[3] += (Ax * gy + Ay * gx) * tf;
    acc.gT[4] += (Ax * gz + Az * gx) * tf;
    acc.gT[5] += (Ay * gz + Az * gy) * tf;
    acc.gV += ux * (Lbb[0] * gx + Lbb[1] * gy + Lbb[2] * gz) +
              uy * (Lbb[3] * gx + Lbb[4] * gy + Lbb[5] * gz) +
              uz * (Lbb[6] * gx + Lbb[7] * gy + Lbb[8] * gz);
    if constexpr (kCorr) {
        const double cx = Mc[0] * rx + Mc[3] * ry + Mc[4] * rz;
        const double cy = Mc[3] * rx + Mc[1] * ry + Mc[5] * rz;
        const double cz = Mc[4] * rx + Mc[5] * ry + Mc[2] * rz;
        const double qx = Mb[0] * rx + Mb[3] * ry + Mb[4] * rz;
        const double qy = Mb[3] * rx + Mb[1] * ry + Mb[5] * rz;
        const double qz = Mb[4] * rx + Mb[5] * ry + Mb[2] * rz;
        const double qc = rx * cx + ry * cy + rz * cz;
        const double qb = rx * qx + ry * qy + rz * qz;
        const double F2 = 2.0 * F;
        const double sG = (Vb * qc + o.Vc * qb) * G;
        acc.gx -= F2 * (Vb * cx + o.Vc * qx) + sG * rx;
        acc.gy -= F2 * (Vb * cy + o.Vc * qy) + sG * ry;
        acc.gz -= F2 * (Vb * cz + o.Vc * qz) + sG * rz;
        acc.gV -= F * qb;
    }
}

__device__ inline AdjOwn adj_own(const double *rec, const AdjRec &ad, int64_t s) {
    AdjOwn o;
    const double2 *ra = rec2(rec, s);
    const double2 p0 = ra[0], p1 = ra[1], p2 = ra[2], p3 = ra[3], p4 = ra[4], p5 = ra[5],
                  p6 = ra[6], p7 = ra[7];
    o.xc = p0.x; o.yc = p0.y; o.zc = p1.x; o.vxc = p1.y; o.vyc = p2.x; o.vzc = p2.y;
    o.rc = p3.x; o.Vc = p3.y; o.mc = p7.x;
    o.Tc[0] = p4.x; o.Tc[1] = p4.y; o.Tc[2] = p5.x; o.Tc[3] = p5.y; o.Tc[4] = p6.x; o.Tc[5] = p6.y;
    const double2 *qa = reinterpret_cast<const double2 *>(ad.arec + s * kAdj);
    const double2 q0 = qa[0], q1 = qa[1], q2 = qa[2], q3 = qa[3], q4 = qa[4], q5 = qa[5], q6 = qa[6];
    o.Lbc[0] = q0.x; o.Lbc[1] = q0.y; o.Lbc[2] = q1.x; o.Lbc[3] = q1.y; o.Lbc[4] = q2.x;
    o.Lbc[5] = q2.y; o.Lbc[6] = q3.x; o.Lbc[7] = q3.y; o.Lbc[8] = q4.x;
    o.abx = q4.y; o.aby = q5.x; o.abz = q5.y; o.rsc = q6.x;
    o.cc = fabs(p7.y);
    o.tens = signbit(p7.y);
    return o;
}

// pre stage: T = ((1 - d) f S - p^ I) / rho^2, V = m / rho, pressure, limiter; writes
// the gradients of user particle a; returns the Y0 contribution
template <int kEos = 0>
__device__ inline double adj_pre(const Consts &k, const AdjRec &ad, const AdjOwn &o,
                                 const AdjAcc &acc, int64_t s, int a, const StateDev &st,
                                 const GradDev &out) {
    double S[6] = {st.sxx[a], st.syy[a], st.szz[a], st.sxy[a], st.sxz[a], st.syz[a]};
    const double j2 = j2_of(S);
    const bool limited = 3.0 * j2 > k.Y0sq;
    const double f = limited ? k.Y0sq / (3.0 * j2) : 1.0;
    const double rc = o.rc;
    const double ir2 = 1.0 / (rc * rc);
    const double keep = st.d ? 1.0 - st.d[a] : 1.0;  // 1 - d
    const double *pb = ad.pb + (size_t)s * kPb;
    double grho = pb[0] + acc.grho - acc.gV * o.Vc / rc;
#pragma unroll
    for (int i = 0; i < 6; ++i) grho += acc.gT[i] * (-2.0 * o.Tc[i] / rc);
    const bool cut = kEos != 2 && k.rho_cut > 0.0 && rc / k.rho0 < k.rho_cut;
    double dp = k.c2;  // dp/drho
    double gu = 0.0;   // Tillotson: cotangent of u
    if constexpr (kEos == 1) {
        dp = k.K0 / k.rho0 * pow(rc / k.rho0, k.n_M - 1.0);
        grho += acc.gc * o.cc * (k.n_M - 1.0) / (2.0 * rc);  // dc/drho = c (n - 1) / (2 rho)
    }
    if constexpr (kEos == 2) {
        // c = sqrt(max(D, 0)), D = dp/drho + p / rho^2 dp/du; the jets carry D's partials
        const Jet R{rc, 1.0, 0.0}, U{st.u ? st.u[a] : 0.0, 0.0, 1.0};
        const PDerT<Jet> pd = tillotson_pd(k, R, U);
        const Jet D = pd.dr + pd.p / (R * R) * pd.du;
        dp = pd.dr.v;
        if (D.v > 0.0) {
            const double ic = 0.5 / sqrt(D.v);
            grho += acc.gc * D.r * ic;
            gu += acc.gc * D.u * ic;
        }
        const double slope_u = o.tens ? keep * pd.du.v : pd.du.v;  // dp^/du
        gu += slope_u * (-(acc.gT[0] + acc.gT[1] + acc.gT[2]) * ir2);
    }
    // dp^/drho; below zero pressure the damaged slope (p < 0 iff rho < rho0 for the
    // liquid and Murnaghan equations)
    const bool tens = kEos == 2 ? o.tens : rc < k.rho0;
    const double slope = tens ? keep * dp : dp;
    if (!cut) grho += slope * (-(acc.gT[0] + acc.gT[1] + acc.gT[2]) * ir2);
    double Stb[6], fb = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        Stb[i] = acc.gT[i] * (ir2 * keep) + pb[1 + i];
        fb += Stb[i] * S[i];
    }
    double gS[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) gS[i] = f * Stb[i];
    double y0 = 0.0;
    if (limited) {
        const double Jb = -fb * f / j2;
#pragma unroll
        for (int i = 0; i < 6; ++i) gS[i] += Jb * (i < 3 ? S[i] : 2.0 * S[i]);
        y0 = fb * 2.0 * f / k.Y0;
    }
    const int A = out.accumulate;
    put(out.x, a, acc.gx, A);
    put(out.y, a, acc.gy, A);
    put(out.z, a, acc.gz, A);
    put(out.vx, a, acc.gvx, A);
    put(out.vy, a, acc.gvy, A);
    put(out.vz, a, acc.gvz, A);
    put(out.rho, a, grho, A);
#pragma unroll
    for (int i = 0; i < 6; ++i) put(out.s[i], a, gS[i], A);
    if constexpr (kEos == 2) put(out.u, a, gu, A);
    return y0;
}

// pair stage + pre stage (see the file header); cell-sweep path, and with the
// correction tensor the only path (also over a pair list)
template <bool kCorr, int kEos, bool kAS, bool kXC>
__global__ __launch_bounds__(kBlock) void k_adj_pairs(GridDev g, int64_t n, Consts k,
                                                      const double *__restrict__ rec, StateDev st,
                                                      AdjRec ad, GradDev out) {
    const int64_t s = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    double y0_part = 0.0;
    if (s < n) {
        const AdjOwn o = adj_own(rec, ad, s);
        AdjAcc acc;
        double Mc[6] = {0, 0, 0, 0, 0, 0};
        if (kCorr) {
#pragma unroll
            for (int i = 0; i < 6; ++i) Mc[i] = ad.Mb[i][s];
        }
        double xo[4] = {0, 0, 0, 0};
        if (kXC) {
#pragma unroll
            for (int i = 0; i < 4; ++i) xo[i] = ad.ext[i][s];
        }
        for_each_candidate(g, s, o.xc, o.yc, o.zc, k.reach, [&](int t) {
            const double2 *rb = rec2(rec, t);
            const double2 b0 = rb[0], b1 = rb[1];
            const double d2 = dist2_exact(o.xc, o.yc, o.zc, b0.x, b0.y, b1.x);
            if (!(d2 < k.h2)) return;
            const double2 *qb = reinterpret_cast<const double2 *>(ad.arec + (int64_t)t * kAdj);
            double Mb[6] = {0, 0, 0, 0, 0, 0};
            if (kCorr) {
#pragma unroll
                for (int i = 0; i < 6; ++i) Mb[i] = ad.Mb[i][t];
            }
            double xb[4] = {0, 0, 0, 0};
            if (kXC) {
#pragma unroll
                for (int i = 0; i < 4; ++i) xb[i] = ad.ext[i][t];
            }
            adj_pair<kCorr, kEos, kAS, kXC>(k, o, d2, b0, b1, rb[2], rb[3], rb[4], rb[5], rb[6],
                                            qb[0], qb[1], qb[2], qb[3], qb[4], qb[5], qb[6], acc,
                                            Mc, Mb, xo, xb, kEos == 2 ? rb[7].y : 0.0);
        });
        if (kXC) {  // dx/dt = v + ...
            acc.gvx += xo[1];
            acc.gvy += xo[2];
            acc.gvz += xo[3];
        }
        y0_part = adj_pre<kEos>(k, ad, o, acc, s, io_index(g, s), st, out);
    }
    const double tot = block_sum(y0_part);
    if (threadIdx.x == 0) put(ad.part_y0, blockIdx.x, tot, ad.add_parts);
}

// the same over the frozen pair list: a workgroup of kSplitAdj wavefronts takes one
// block of 64 slots, wavefront q evaluating steps q, q + kSplitAdj, ... (the first seven
// chunks of each partner's two records gathered cooperatively; with Tillotson all eight
// of the forward record, whose last holds the partner's signed sound speed); the
// partial sums are folded into wavefront 0, which runs the pre stage and the Y0 sum.
// With the du and dx/dt cotangents each lane loads its own partner's four (one list
// entry per lane and step)
template <int kEos, bool kAS, bool kXC = false>
__global__ __launch_bounds__(64 * kSplitAdj) void k_adj_pairs_list(GridDev g, int64_t n, Consts k,
                                                                   const double *__restrict__ rec,
                                                                   StateDev st, AdjRec ad,
                                                                   GradDev out) {
    constexpr int kF = kEos == 2 ? 8 : 7;  // forward-record chunks gathered
    __shared__ double2 lbuf[kSplitAdj][64 * (kF + 7)];
    const int q = threadIdx.x >> 6;
    double2 *bf = lbuf[q];
    double2 *ba = bf + 64 * kF;
    auto fchunk = [&](int c) { return kF == 8 ? dma8_chunk(bf, c) : dma_chunk<7>(bf, c); };
    const int64_t w = xcd_block(gridDim.x);
    const int64_t w0 = w * 64;
    if (w0 >= n) return;  // whole workgroup past the end
    const int64_t s = w0 + __lane_id();
    const bool act = s < n;
    const int64_t base = g.pl_block[w];
    const int cnt = act ? g.pl_count[s] : 0;
    const int steps = list_steps(cnt);
    const AdjOwn o = adj_own(rec, ad, act ? s : w0);
    AdjAcc acc;
    double xo[4] = {0, 0, 0, 0};
    if constexpr (kXC) {
#pragma unroll
        for (int i = 0; i < 4; ++i) xo[i] = ad.ext[i][act ? s : w0];
    }
    const char *rf = reinterpret_cast<const char *>(rec);
    const char *ra = reinterpret_cast<const char *>(ad.arec);
    const int32_t *row = g.pl_slot + base + __lane_id();
    // One step ahead: the gathers of step j + kSplitAdj are in flight while step j is
    // evaluated.  Each lane reads its step-j chunks into registers, the wavefront
    // syncs, and only then are the buffers refilled.
    auto gather = [&](int e) {
        if constexpr (kF == 8)
            gather_dma8(rf, kRec * 8, e, bf);
        else
            gather_dma<7>(rf, kRec * 8, e, bf);
        gather_dma<7>(ra, kAdj * 8, e, ba);
    };
    int cur = q < steps ? row[(int64_t)q << 6] : 0;  // this lane's partner slot of step j
    if (q < steps) gather(cur);
    int nxt = q + kSplitAdj < steps ? row[(int64_t)(q + kSplitAdj) << 6] : 0;
    for (int j = q; j < steps; j += kSplitAdj) {
        wait_vm();
        const double2 b0 = fchunk(0), b1 = fchunk(1), b2 = fchunk(2), b3 = fchunk(3),
                      b4 = fchunk(4), b5 = fchunk(5), b6 = fchunk(6);
        const double cb = kF == 8 ? fchunk(7).y : 0.0;
        const double2 q0 = dma_chunk<7>(ba, 0), q1 = dma_chunk<7>(ba, 1),
                      q2 = dma_chunk<7>(ba, 2), q3 = dma_chunk<7>(ba, 3),
                      q4 = dma_chunk<7>(ba, 4), q5 = dma_chunk<7>(ba, 5),
                      q6 = dma_chunk<7>(ba, 6);
        wave_sync();
        const int mine = cur;
        if (j + kSplitAdj < steps) {
            gather(nxt);
            cur = nxt;
            if (j + 2 * kSplitAdj < steps) nxt = row[(int64_t)(j + 2 * kSplitAdj) << 6];
        }
        if (j < cnt) {
            const double d2 = dist2_exact(o.xc, o.yc, o.zc, b0.x, b0.y, b1.x);
            double xb[4] = {0, 0, 0, 0};
            if constexpr (kXC) {
#pragma unroll
                for (int i = 0; i < 4; ++i) xb[i] = ad.ext[i][mine];
            }
            if (d2 < k.h2)
                adj_pair<false, kEos, kAS, kXC>(k, o, d2, b0, b1, b2, b3, b4, b5, b6, q0, q1,
                                                q2, q3, q4, q5, q6, acc, nullptr, nullptr, xo,
                                                xb, cb);
        }
    }
    fold_adj<kSplitAdj, kSplitAdj * 64 * (kF + 7) * 2>(acc, reinterpret_cast<double *>(lbuf));
    if (q != 0) return;
    if constexpr (kXC) {  // dx/dt = v + ...
        acc.gvx += xo[1];
        acc.gvy += xo[2];
        acc.gvz += xo[3];
    }
    double y0_part = act ? adj_pre<kEos>(k, ad, o, acc, s, io_index(g, s), st, out) : 0.0;
    // fixed-order wavefront sum
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) y0_part += __shfl_xor(y0_part, off);
    if (__lane_id() == 0) put(ad.part_y0, (int)w, y0_part, ad.add_parts);
}

}  // namespace

namespace {
// Sum of p[threadIdx.x + kBlock k] over k in a fixed order: eight running sums (k mod 8)
// so that eight loads are in flight, added pairwise at the end.
__device__ inline double strided_sum(const double *__restrict__ p, int64_t m) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = threadIdx.x; i < m; i += 8 * kBlock) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t j = i + (int64_t)u * kBlock;
            if (j < m) a[u] += p[j];
        }
    }
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// one block: dparams[i] (+)= sum of part_i in a fixed order (a null part is skipped)
__global__ __launch_bounds__(kBlock) void k_reduce_params(const double *__restrict__ p0,
                                                          int64_t m0,
                                                          const double *__restrict__ p1,
                                                          int64_t m1, double *dparams,
                                                          int accumulate) {
    double a = p0 ? strided_sum(p0, m0) : 0.0, b = p1 ? strided_sum(p1, m1) : 0.0;
    a = block_sum(a);
    b = block_sum(b);
    if (threadIdx.x == 0) {
        if (accumulate) {
            if (p0) dparams[0] += a;
            if (p1) dparams[1] += b;
        } else {
            dparams[0] = a;
            dparams[1] = b;
        }
    }
}

}  // namespace

int reduce_params_launch(const double *p0, int64_t m0, const double *p1, int64_t m1,
                         double *dparams, int accumulate, hipStream_t s) {
    k_reduce_params<<<1, kBlock, 0, s>>>(p0, m0, p1, m1, dparams, accumulate);
    SPH_LAUNCHED();
    return SPH_OK;
}

size_t adjoint_ws_bytes(int64_t n) {
    Carve c(nullptr);
    c.take<double>((size_t)n * kRec);
    carve_adj(c, n);
    return c.used;
}

CotDev cot_dev(const sph_deriv_cot *c) {
    return CotDev{c->ax, c->ay, c->az, c->drho, {c->dsxx, c->dsyy, c->dszz, c->dsxy, c->dsxz, c->dsyz},
                  c->rho_sum, c->du, {c->dx, c->dy, c->dz}};
}

GradDev grad_dev(const sph_fields *g, int accumulate) {
    return GradDev{g->x, g->y, g->z, g->vx, g->vy, g->vz, g->rho,
                   {g->sxx, g->syy, g->szz, g->sxy, g->sxz, g->syz}, accumulate, g->u};
}

// Adjoint of one right-hand side on a carved workspace; gradients written or
// accumulated (accumulate != 0) into grad; dparams written or accumulated.
int rhs_adjoint_launch(const sph_grid *grid, const sph_state *state, const sph_params *params,
                       const CotDev &cot, const GradDev &grad, double *dparams, int accumulate_params,
                       Carve &c, hipStream_t s, const double *L_in, bool slot_state,
                       double *acc_parts, bool post_ready, const double *rec_in) {
    const int64_t n = grid->n;
    GridDev g = grid_dev(grid);
    if (slot_state) g.io = nullptr;
    Consts k = make_consts(*params, g.delta);
    const AdjBuffers bufs = adj_buffers(c, n);
    double *rec = bufs.rec;
    AdjRec ad = bufs.ad;
    if (acc_parts) {
        ad.part_mu = acc_parts;
        ad.part_y0 = acc_parts + blocks_for(n);
        ad.add_parts = 1;
    }
    StateDev st = state_dev(state);
    int rc;
    if (post_ready) {
        if (!L_in || !acc_parts) return fail(SPH_ERR_INVALID_ARG, "post stage not prepared");
    } else if (rec_in) {
        rec = const_cast<double *>(rec_in);  // the forward's records (read only)
        if ((rc = invert_launch(g, n, ad.inv, s))) return rc;
    } else if ((rc = prepass_launch(g, st, n, k, rec, c.status(), s, nullptr, ad.inv))) {
        return rc;
    }
    ad.lw = vgrad_width(k.corr);
    if (L_in) {
        ad.L = const_cast<double *>(L_in);
    } else {
        TimedRegion t("adjoint_L", s);
        const dim3 gb(blocks_for(n)), tb(kBlock);
        const dim3 gl(blocks_for(n, 64)), tl(64 * kSplit);
        if (g.pl_count && k.corr)
            k_adj_L_list<true><<<gl, tl, 0, s>>>(g, n, k, rec, ad);
        else if (g.pl_count)
            k_adj_L_list<false><<<gl, tl, 0, s>>>(g, n, k, rec, ad);
        else if (k.corr)
            k_adj_L<true><<<gb, tb, 0, s>>>(g, n, k, rec, ad);
        else
            k_adj_L<false><<<gb, tb, 0, s>>>(g, n, k, rec, ad);
        SPH_LAUNCHED();
    }
    if (!post_ready) {
        // the prepass (or invert_launch) filled ad.inv when the state is in user order
        k_adj_post<<<blocks_for(n), kBlock, 0, s>>>(g, n, k, rec, st, cot, ad,
                                                    g.io ? ad.inv : nullptr);
        SPH_LAUNCHED();
    }
    {
        TimedRegion t("adjoint_pairs", s);
        const bool as = k.eps_s > 0.0;
        const bool xc = cot.du || cot.dx[0] || cot.dx[1] || cot.dx[2];
        auto launch = [&](auto eos_t, auto as_t) {
            constexpr int E = decltype(eos_t)::value;
            constexpr bool A = decltype(as_t)::value;
            const dim3 gb(blocks_for(n)), tb(kBlock);
            if (xc && k.corr)
                k_adj_pairs<true, E, A, true><<<gb, tb, 0, s>>>(g, n, k, rec, st, ad, grad);
            else if (xc && g.pl_count)
                k_adj_pairs_list<E, A, true><<<blocks_for(n, 64), 64 * kSplitAdj, 0, s>>>(g, n, k, rec, st, ad, grad);
            else if (xc)
                k_adj_pairs<false, E, A, true><<<gb, tb, 0, s>>>(g, n, k, rec, st, ad, grad);
            else if (k.corr)
                k_adj_pairs<true, E, A, false><<<gb, tb, 0, s>>>(g, n, k, rec, st, ad, grad);
            else if (g.pl_count)
                k_adj_pairs_list<E, A><<<blocks_for(n, 64), 64 * kSplitAdj, 0, s>>>(g, n, k, rec, st, ad, grad);
            else
                k_adj_pairs<false, E, A, false><<<gb, tb, 0, s>>>(g, n, k, rec, st, ad, grad);
        };
        using T = std::true_type;
        using F = std::false_type;
        using E0 = std::integral_constant<int, 0>;
        using E1 = std::integral_constant<int, 1>;
        using E2 = std::integral_constant<int, 2>;
        if (k.eos == 2)
            as ? launch(E2{}, T{}) : launch(E2{}, F{});
        else if (k.eos == 1)
            as ? launch(E1{}, T{}) : launch(E1{}, F{});
        else
            as ? launch(E0{}, T{}) : launch(E0{}, F{});
        SPH_LAUNCHED();
    }
    if (acc_parts) return SPH_OK;  // the caller reduces its accumulators
    const bool per_wave = g.pl_count && !k.corr;
    const int64_t m_y0 = per_wave ? blocks_for(n, 64) : blocks_for(n);
    return reduce_params_launch(ad.part_mu, blocks_for(n), ad.part_y0, m_y0, dparams,
                                accumulate_params, s);
}

int check_grad(const sph_fields *g) {
    if (!g) return fail(SPH_ERR_INVALID_ARG, "gradient struct is NULL");
    const double *p[] = {g->x, g->y, g->z, g->vx, g->vy, g->vz, g->rho,
                         g->sxx, g->syy, g->szz, g->sxy, g->sxz, g->syz};
    for (const double *q : p)
        if (!q) return fail(SPH_ERR_INVALID_ARG, "gradient array is NULL");
    return SPH_OK;
}

}  // namespace sph

using namespace sph;

extern "C" int sph_rhs_adjoint(const sph_grid *grid, const sph_state *state,
                               const sph_params *params, const sph_deriv_cot *cot,
                               const sph_state_grad *grad, double *dparams, void *ws,
                               size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_state(grid, state)) ||
        (rc = check_params(grid, params)) || (rc = check_grad(grad)))
        return rc;
    if (!cot) return fail(SPH_ERR_INVALID_ARG, "cotangent struct is NULL");
    if (!dparams || !ws) return fail(SPH_ERR_INVALID_ARG, "null pointer");
    if (params->eos == 2.0 && !grad->u)
        return fail(SPH_ERR_INVALID_ARG, "the Tillotson adjoint writes the gradient of u: grad->u is NULL");
    const size_t need = adjoint_ws_bytes(grid->n);
    if (ws_bytes < need) return fail(SPH_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = clear_status(ws, s))) return rc;
    Carve c(ws);
    return rhs_adjoint_launch(grid, state, params, cot_dev(cot), grad_dev(grad, 0), dparams, 0, c, s,
                              cot->vgrad, false, nullptr, false, cot->rec);
}
