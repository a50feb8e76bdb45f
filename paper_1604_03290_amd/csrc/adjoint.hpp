// Internals of the right-hand side's adjoint shared by adjoint.hip and the
// leapfrog's reverse sweep (which fuses the post stage into its kick pass).
#pragma once

#include "common.hpp"
#include "rhs_common.hpp"

namespace sph {

// Adjoint operand records, one 128-byte record per slot (seven chunks used):
//   Lbar(9) | abar(3) | rho_sum bar | - - -
constexpr int kAdj = 16;

// Per-slot records of the post stage's partial cotangents: the density's, then that of
// f_Y S from the rotation terms (stored components); one 64-byte record per slot.
constexpr int kPb = 8;

struct AdjRec {
    double *L;         // forward velocity gradient and, with the correction, moment matrix
                       // (slot order, vgrad_width(corr) values per slot)
    int lw;            // values per slot of L
    double *Mb[6];     // with the correction: its cotangent, symmetrised
    double *arec;      // adjoint records [n][kAdj]
    double *pb;        // partial cotangents [n][kPb]: rho, then S~ (6)
    double *part_mu;   // per-block partial sums (ceil(n / 256))
    double *part_y0;   // per block, or per wavefront for the list kernel (ceil(n / 64))
    double *ext[4];    // cotangents of du and dx/dt (slot order), when given
    int32_t *inv;      // slot of every user index (the inverse of the grid's perm)
    int add_parts;     // add the block sums to part_* instead of writing them
};

inline AdjRec carve_adj(Carve &c, int64_t n) {
    AdjRec r;
    r.L = c.take<double>((size_t)n * vgrad_width(true));
    r.lw = vgrad_width(false);
    for (int i = 0; i < 6; ++i) r.Mb[i] = c.take<double>(n);
    r.arec = c.take<double>((size_t)n * kAdj);
    r.pb = c.take<double>((size_t)n * kPb);
    r.part_mu = c.take<double>(blocks_for(n));
    r.part_y0 = c.take<double>(blocks_for(n, 64));
    for (int i = 0; i < 4; ++i) r.ext[i] = c.take<double>(n);
    r.inv = c.take<int32_t>(n);
    r.add_parts = 0;
    return r;
}

// The operand records and adjoint buffers of rhs_adjoint_launch, its first carves.
struct AdjBuffers {
    double *rec;
    AdjRec ad;
};

inline AdjBuffers adj_buffers(Carve &c, int64_t n) {
    AdjBuffers b;
    b.rec = c.take<double>((size_t)n * kRec);
    b.ad = carve_adj(c, n);
    return b;
}

// Post stage at slot s (see adjoint.hip's header): from the forward velocity
// gradient L (row-major), density rho and stress S (before the limiter) of the
// particle and the cotangents of its outputs (c6: stored dS components, rdot:
// drho, ax..az: acceleration, rs_cot: rho_sum), writes the adjoint record, the
// partial density cotangent and the rotation terms' stress cotangent; returns
// the particle's mu contribution.
//
// With the correction tensor (corr; Mv: the moment matrix) the strain and
// rotation rates see Lc = L C, C = M^-1 (section 3.1.6), so with Lcbar their
// cotangent:  Lbar = Lcbar C^T - rho drho_bar I,  Cbar = L^T Lcbar and
// Mbar = -C^T Cbar C^T, stored symmetrised in ad.Mb (zero where C fell back to
// the identity); mu_bar and S~_bar use Lc.
__device__ inline double adj_post_at(const Consts &k, int64_t s, const double Lv[9], bool corr,
                                     const double Mv[6], double rho, const double S[6],
                                     const double c6[6], double rdot, double ax, double ay,
                                     double az, double rs_cot, const AdjRec &ad) {
    double L[3][3], C[9];
    const bool inv = corr ? correction_tensor(Mv, C) : false;
    if (corr) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                L[i][j] = Lv[3 * i] * C[j] + Lv[3 * i + 1] * C[3 + j] + Lv[3 * i + 2] * C[6 + j];
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) L[i / 3][i % 3] = Lv[i];
    }
    const double f = yield_factor(k, S);
    const double St[3][3] = {{f * S[0], f * S[3], f * S[4]},
                             {f * S[3], f * S[1], f * S[5]},
                             {f * S[4], f * S[5], f * S[2]}};
    const double G[3][3] = {{c6[0], 0.5 * c6[3], 0.5 * c6[4]},
                            {0.5 * c6[3], c6[1], 0.5 * c6[5]},
                            {0.5 * c6[4], 0.5 * c6[5], c6[2]}};
    const double trG = G[0][0] + G[1][1] + G[2][2];
    double R[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) R[i][j] = 0.5 * (L[i][j] - L[j][i]);
    double Lb[9];
    double mu_b = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double D = G[i][j] - (i == j ? trG / 3.0 : 0.0);
            double P = 0.0;  // (G S~ - S~ G)_ij
#pragma unroll
            for (int m = 0; m < 3; ++m) P += G[i][m] * St[m][j] - St[i][m] * G[m][j];
            Lb[3 * i + j] = corr ? 2.0 * k.mu * D + P : (i == j ? -rho * rdot : 0.0) + 2.0 * k.mu * D + P;
            mu_b += 2.0 * D * L[i][j];
        }
    if (corr) {
        // Lb holds Lcbar here
        double Cb[9], T[9], Mb[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Cb[3 * i + j] = Lv[i] * Lb[j] + Lv[3 + i] * Lb[3 + j] + Lv[6 + i] * Lb[6 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                T[3 * i + j] = Cb[3 * i] * C[3 * j] + Cb[3 * i + 1] * C[3 * j + 1] + Cb[3 * i + 2] * C[3 * j + 2];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Mb[3 * i + j] = -(C[i] * T[j] + C[3 + i] * T[3 + j] + C[6 + i] * T[6 + j]);
        const double z = inv ? 1.0 : 0.0;
        ad.Mb[0][s] = z * Mb[0];
        ad.Mb[1][s] = z * Mb[4];
        ad.Mb[2][s] = z * Mb[8];
        ad.Mb[3][s] = z * 0.5 * (Mb[1] + Mb[3]);
        ad.Mb[4][s] = z * 0.5 * (Mb[2] + Mb[6]);
        ad.Mb[5][s] = z * 0.5 * (Mb[5] + Mb[7]);
        double Lu[9];  // Lcbar C^T
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Lu[3 * i + j] = Lb[3 * i] * C[3 * j] + Lb[3 * i + 1] * C[3 * j + 1] + Lb[3 * i + 2] * C[3 * j + 2];
#pragma unroll
        for (int i = 0; i < 9; ++i) Lb[i] = Lu[i] + (i % 4 == 0 ? -rho * rdot : 0.0);
    }
    double *pb = ad.pb + (size_t)s * kPb;
    pb[0] = -(Lv[0] + Lv[4] + Lv[8]) * rdot;
    double Sb[3][3];  // G R - R G
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < 3; ++m) v += G[i][m] * R[m][j] - R[i][m] * G[m][j];
            Sb[i][j] = v;
        }
    pb[1] = Sb[0][0];
    pb[2] = Sb[1][1];
    pb[3] = Sb[2][2];
    pb[4] = Sb[0][1] + Sb[1][0];
    pb[5] = Sb[0][2] + Sb[2][0];
    pb[6] = Sb[1][2] + Sb[2][1];
    pb[7] = 0.0;
    double2 *o = reinterpret_cast<double2 *>(ad.arec + s * kAdj);
    o[0] = make_double2(Lb[0], Lb[1]);
    o[1] = make_double2(Lb[2], Lb[3]);
    o[2] = make_double2(Lb[4], Lb[5]);
    o[3] = make_double2(Lb[6], Lb[7]);
    o[4] = make_double2(Lb[8], ax);
    o[5] = make_double2(ay, az);
    o[6] = make_double2(rs_cot, 0.0);
    o[7] = make_double2(0.0, 0.0);
    return mu_b;
}

}  // namespace sph
