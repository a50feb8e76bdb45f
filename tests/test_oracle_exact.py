"""Exact pins of the oracle: values fixed by the paper's definitions, evaluated in exact
rational arithmetic or in closed form, that the oracle's floating-point code must meet
to rounding.

  viscosity   section 3.1.3 (eq. accel_artvisc): two particles approaching head-on
              feel only the artificial viscosity; its acceleration derived in one
              dimension along their line, with the pair's mean density (rho_a +
              rho_b) / 2, h_ab = h and the eps h^2 term, in exact rationals
  whole RHS   sections 2.2-2.6, 3.1: four particles at the corners of an Euler brick
              (every distance between them rational) and one isolated particle;
              density sum, velocity gradient, acceleration with pressure, limited
              deviator and viscosity, continuity sum and Hooke + Jaumann stress rate,
              all in exact rationals
  lattice     eq. density_by_kernel_sum and section 3.1.6 on an unjittered cubic
              lattice at h = 2.4 dx: rho_sum / rho0 = 1.0008095 and the gradient
              factor kappa = 0.98169 from integer-vector sums, with the cubic spline
              written in its half-support form (Monaghan's M4 with H = h / 2)
  Tillotson   section 2.5.3: the expanded form's ideal-gas limit p = a rho u and
              c^2 = a (1 + a) u far below rho0, and the compressed form's hot value
              p = (a + b / (1 + u / E0)) rho0 u at rho = rho0

Every value below that the kernel's normalisation multiplies carries the factor
s = 8 / pi once; it is kept symbolic (the rational part is exact) and applied in
floating point at the end.
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import workloads as W
from oracle import native

SIGMA = 8.0 / math.pi  # the 3-D normalisation of the cubic spline (section 3.1.1)


def params(h, **over):
    p = W.MATERIAL.copy()
    p.update(h=float(h), dmpd=float(h) / 2.4)
    p.update(over)
    return np.array([p[k] for k in W.PARAM_ORDER], dtype=np.float64)


# ------------------------------------------------------------ exact rationals --
def exact_sqrt(x: Fr) -> Fr:
    """Square root of a rational that is the square of a rational."""
    n, d = math.isqrt(x.numerator), math.isqrt(x.denominator)
    assert Fr(n * n, d * d) == x, "distance is not rational"
    return Fr(n, d)


def spline(q: Fr):
    """Shape w(q) of W = s / h^3 w and its derivative dw/dq (section 3.1.1)."""
    if q < Fr(1, 2):
        return 6 * q ** 3 - 6 * q ** 2 + 1, 18 * q ** 2 - 12 * q
    if q < 1:
        return 2 * (1 - q) ** 3, -6 * (1 - q) ** 2
    return Fr(0), Fr(0)


def F(a):
    return [Fr(float(v)) for v in a]


def exact_rhs(pos, vel, rho, S, m, h, rho0, c, mu, Y0, alpha, beta, eps):
    """Every output of the right-hand side in exact rationals, each as the coefficient of
    s = 8 / pi.  pos, vel (3, n), S (6, n) xx yy zz xy xz yz, floats that are exact
    dyadic rationals."""
    n = len(rho)
    X = [F(pos[:, a]) for a in range(n)]
    V = [F(vel[:, a]) for a in range(n)]
    R = F(rho)
    M = F(m)
    h, rho0, c, mu, Y0, alpha, beta, eps = map(lambda v: Fr(float(v)),
                                               (h, rho0, c, mu, Y0, alpha, beta, eps))
    ij = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]

    def tensor(s6):
        t = [[Fr(0)] * 3 for _ in range(3)]
        for (i, j), v in zip(ij, s6):
            t[i][j] = t[j][i] = v
        return t

    Smat, fY, T = [], [], []
    for a in range(n):
        s6 = F(S[:, a])
        St = tensor(s6)
        J2 = sum(St[i][j] ** 2 for i in range(3) for j in range(3)) / 2  # S:S / 2
        f = min(Y0 ** 2 / (3 * J2), Fr(1)) if J2 > 0 else Fr(1)  # section 2.6
        p = c ** 2 * (R[a] - rho0)  # section 2.5.1
        sig = [[f * St[i][j] - (p if i == j else 0) for j in range(3)] for i in range(3)]
        Smat.append(St)
        fY.append(f)
        T.append([[sig[i][j] / R[a] ** 2 for j in range(3)] for i in range(3)])

    out = {k: [] for k in ("acc", "drho", "dS", "rho_sum", "L")}
    approaching = receding = 0
    for a in range(n):
        rs = M[a] * spline(Fr(0))[0] / h ** 3  # own term m_a W(0)
        L = [[Fr(0)] * 3 for _ in range(3)]
        acc = [Fr(0)] * 3
        drho = Fr(0)
        for b in range(n):
            if b == a:
                continue
            r = [X[a][i] - X[b][i] for i in range(3)]  # x_a - x_b
            d2 = sum(v * v for v in r)
            if not d2 < h * h:  # section 3.5.2: partners closer than h
                continue
            d = exact_sqrt(d2)
            wq, dwq = spline(d / h)
            rs += M[b] * wq / h ** 3
            g = [dwq / h ** 4 * r[i] / d for i in range(3)]  # grad_a W_ab / s
            Vb = M[b] / R[b]
            dv = [V[b][i] - V[a][i] for i in range(3)]
            for i in range(3):
                for j in range(3):
                    L[i][j] += Vb * dv[i] * g[j]
            w = -sum(dv[i] * r[i] for i in range(3))  # (v_a - v_b) . (x_a - x_b)
            Pi = Fr(0)
            if w < 0:  # section 3.1.3: approaching pairs only
                nu = h * w / (d2 + eps * h * h)
                Pi = (-alpha * c * nu + beta * nu * nu) / ((R[a] + R[b]) / 2)
                approaching += 1
            else:
                receding += 1
            for i in range(3):
                acc[i] += M[b] * sum((T[a][i][j] + T[b][i][j] - (Pi if i == j else 0)) * g[j]
                                     for j in range(3))
            drho += R[a] * Vb * sum(-dv[i] * g[i] for i in range(3))  # eq. continuity_equation_sph
        ed = [[(L[i][j] + L[j][i]) / 2 for j in range(3)] for i in range(3)]
        Rt = [[(L[i][j] - L[j][i]) / 2 for j in range(3)] for i in range(3)]
        tr = ed[0][0] + ed[1][1] + ed[2][2]
        St = [[fY[a] * Smat[a][i][j] for j in range(3)] for i in range(3)]
        dS = [[2 * mu * (ed[i][j] - (tr / 3 if i == j else 0))
               + sum(Rt[i][k] * St[k][j] - St[i][k] * Rt[k][j] for k in range(3))
               for j in range(3)] for i in range(3)]
        out["acc"].append(acc)
        out["drho"].append(drho)
        out["dS"].append([dS[i][j] for i, j in ij])
        out["rho_sum"].append(rs)
        out["L"].append([L[i][j] for i in range(3) for j in range(3)])
    res = {k: SIGMA * np.array([[float(x) for x in v] if isinstance(v, list) else float(v)
                                for v in vals], dtype=np.float64).T
           for k, vals in out.items()}
    return res, approaching, receding


def close(got, want, tol):
    scale = np.abs(want).max()
    assert scale > 0
    return np.abs(got - want).max() <= tol * scale


# --------------------------------------------------- viscosity, two particles --
@pytest.mark.parametrize("k", [32, 16])  # distance 13/32 (inner spline piece), 13/16 (outer)
def test_head_on_viscous_acceleration_closed_form(k):
    # a at the origin, b at distance d along e = (3, 4, 12) / 13; a moves towards b at
    # 6.5, b towards a at 3.25.  Zero pressure (rho < rho0 under a tension cut-off of 1)
    # and zero deviator: only the viscosity acts.  In one dimension along e, with
    # w = -(u_a - u_b) d, nu = h w / (d^2 + eps h^2), Pi = (-alpha c nu + beta nu^2) /
    # ((rho_a + rho_b) / 2), the bracket's -Pi I pushes the two apart:
    #   a_a = -m_b Pi |W'(d)| e,   a_b = +m_a Pi |W'(d)| e.
    h, d = Fr(1), Fr(13, k)
    e = np.array([3.0, 4.0, 12.0]) / 13.0
    xb = np.array([3.0, 4.0, 12.0]) / k
    va, vb = np.array([3.0, 4.0, 12.0]) / 2, -np.array([3.0, 4.0, 12.0]) / 4
    rho, m = (2500.0, 2000.0), (0.75, 1.25)
    alpha, beta, eps, c = Fr(1, 2), Fr(3, 2), Fr(1, 64), Fr(5000)
    wv = W.two_particles((0, 0, 0), xb, va, vb, rho, None, m, h=1.0, alpha=0.5, beta=1.5,
                         eps_v=1 / 64, rho_cut=1.0)
    got = native.rhs_workload(wv)["acc"]
    u_rel = Fr(13, 2) + Fr(13, 4)
    w = -u_rel * d
    nu = h * w / (d * d + eps * h * h)
    Pi = (-alpha * c * nu + beta * nu * nu) / ((Fr(2500) + Fr(2000)) / 2)
    assert Pi > 0
    dW = abs(spline(d / h)[1]) / h ** 4  # |W'(d)| / s
    want_a = -float(Fr(5, 4) * Pi * dW) * SIGMA * e
    want_b = float(Fr(3, 4) * Pi * dW) * SIGMA * e
    assert np.abs(got[:, 0] - want_a).max() <= 1e-14 * np.abs(want_a).max()
    assert np.abs(got[:, 1] - want_b).max() <= 1e-14 * np.abs(want_b).max()


# ------------------------------------------------------ whole right-hand side --
def brick_set():
    # corners O, (44, 0, 0), (0, 117, 0), (0, 0, 240) of the Euler brick (face
    # diagonals 125, 244, 267) in units of 1/512, shifted; a fifth particle far away
    base = np.array([[0, 44, 0, 0], [0, 0, 117, 0], [0, 0, 0, 240]], dtype=np.float64) / 512
    pos = np.concatenate([base + np.array([[0.25], [0.5], [0.125]]), [[2.0], [2.0], [2.0]]], 1)
    vel = np.array([[3.0, -2.0, 1.25, 0.75, 1.0],
                    [-1.5, 0.5, 2.5, -0.25, 1.0],
                    [0.25, 1.0, -3.0, 2.0, 1.0]]) * 8.0
    rho = np.array([2690.0, 2710.0, 2725.0, 2680.0, 2700.0])
    S = np.array([[2e8, 1e7, -5e7, 0.0, 4e6],
                  [-1e8, 2e7, 2.5e7, 0.0, -2e6],
                  [-1e8, -3e7, 2.5e7, 0.0, -2e6],
                  [5e7, 4e6, 1.25e7, 0.0, 1e6],
                  [0.0, -5e6, 6.25e6, 0.0, 0.0],
                  [2.5e7, 6e6, -3.125e6, 0.0, 5e5]])
    m = np.array([0.5, 0.75, 1.0, 1.25, 1.5])
    return pos, vel, rho, S, m


def test_whole_rhs_of_a_small_set_in_exact_rationals():
    pos, vel, rho, S, m = brick_set()
    h = 300.0 / 512  # every brick distance inside h: q from 0.15 to 0.89, both spline pieces
    pv = params(h, alpha=0.5, beta=1.5, eps_v=1 / 64)
    exact, n_app, n_rec = exact_rhs(pos, vel, rho, S, m, h, 2700.0, 5000.0, 2.7e10, 3e8,
                                    0.5, 1.5, 1 / 64)
    assert n_app > 0 and n_rec > 0  # both sides of the viscosity switch
    got = native.rhs(pos, vel, rho, S, m, pv)
    for k, tol in (("rho_sum", 1e-15), ("L", 1e-14), ("acc", 1e-14), ("drho", 1e-14),
                   ("dS", 1e-13)):
        assert close(got[k], exact[k], tol), k
    # the isolated particle: its own density term only, nothing else
    assert abs(got["rho_sum"][4] - exact["rho_sum"][4]) <= 1e-15 * exact["rho_sum"][4]
    assert np.all(got["acc"][:, 4] == 0.0) and np.all(got["L"][:, 4] == 0.0)
    # particle 0's deviator is limited (3 J2 > Y0^2), the others are not
    J2 = 0.5 * (S[0] ** 2 + S[1] ** 2 + S[2] ** 2) + S[3] ** 2 + S[4] ** 2 + S[5] ** 2
    assert 3 * J2[0] > 9e16 and np.all(3 * J2[1:] < 9e16)


def test_exact_rhs_is_sensitive_to_each_guarded_factor():
    # the same comparison fails when a constant of the definition is off by 1 %: eps of
    # the eps h^2 term, alpha, beta, the sound speed, the shear modulus, and the kernel
    # normalisation (the mean density in Pi is pinned by the head-on closed form)
    pos, vel, rho, S, m = brick_set()
    h = 300.0 / 512
    got = native.rhs(pos, vel, rho, S, m, params(h, alpha=0.5, beta=1.5, eps_v=1 / 64))
    base = (pos, vel, rho, S, m, h, 2700.0, 5000.0, 2.7e10, 3e8, 0.5, 1.5, 1 / 64)
    for i, f in ((12, 1.01), (10, 1.01), (7, 1.01), (8, 1.01), (11, 1.01)):
        args = list(base)
        args[i] = args[i] * f
        off = exact_rhs(*args)[0]
        assert not all(close(got[k], off[k], 1e-12) for k in ("acc", "dS")), i
    off = exact_rhs(*base)[0]
    assert not close(got["rho_sum"], 1.01 * off["rho_sum"], 1e-12)


# ------------------------------------------------------------- lattice sums --
def m4(r, H):
    """Cubic B-spline in Monaghan's half-support form, W = 1 / (pi H^3) f(r / H) with
    f = 1 - 3/2 s^2 + 3/4 s^3 (s < 1), (2 - s)^3 / 4 (1 <= s < 2), and dW/dr."""
    s = r / H
    f = np.where(s < 1, 1 - 1.5 * s ** 2 + 0.75 * s ** 3, np.where(s < 2, 0.25 * (2 - s) ** 3, 0.0))
    df = np.where(s < 1, -3 * s + 2.25 * s ** 2, np.where(s < 2, -0.75 * (2 - s) ** 2, 0.0))
    return f / (math.pi * H ** 3), df / (math.pi * H ** 4)


def lattice_vectors():
    return np.array([v for v in itertools.product(range(-3, 4), repeat=3)], dtype=np.float64)


def lattice_density_ratio():
    # rho_sum / rho0 = sum over lattice vectors n (self included) of dx^3 W(|n| dx)
    n = lattice_vectors()
    Wv, _ = m4(np.sqrt((n ** 2).sum(1)), 1.2)  # dx = 1, h = 2.4, H = h / 2
    return Wv.sum()


def lattice_gradient_factor():
    # L = A sum_n dx^3 (n dx) (x) grad_a W = kappa A with, by cubic symmetry,
    # kappa = -(1/3) sum_n |n| dW/dr (|n|)  (dx = 1)
    n = lattice_vectors()
    r = np.sqrt((n ** 2).sum(1))
    _, dW = m4(r, 1.2)
    return -(r * dW).sum() / 3.0


def lattice(n_side=9, dx=0.1):
    return W.cube(n_side, dx, seed=1, jitter=0.0, state="rest", h_over_dx=2.4)


def interior(n_side, margin=3):
    idx = np.arange(n_side ** 3)
    ix, iy, iz = idx % n_side, (idx // n_side) % n_side, idx // (n_side * n_side)
    ok = np.ones(idx.size, bool)
    for t in (ix, iy, iz):
        ok &= (t >= margin) & (t <= n_side - 1 - margin)
    return idx[ok]


def test_lattice_density_sum_exact_value():
    ratio = lattice_density_ratio()
    assert abs(ratio - 1.0008095) < 5e-8
    w = lattice(9)
    got = native.rhs_workload(w)["rho_sum"][interior(9)] / w.params["rho0"]
    assert np.abs(got - ratio).max() <= 1e-13


def test_lattice_gradient_factor_exact_value():
    kappa = lattice_gradient_factor()
    assert abs(kappa - 0.98169) < 5e-6
    w = lattice(9)
    A = np.array([[30.0, -20.0, 10.0], [5.0, 40.0, -15.0], [-25.0, 35.0, 20.0]])
    w.vel = np.ascontiguousarray(A @ w.pos)
    L = native.rhs_workload(w)["L"].reshape(3, 3, -1)[:, :, interior(9)]
    assert np.abs(L - kappa * A[:, :, None]).max() <= 1e-12 * np.abs(A).max()


# ---------------------------------------------------------------- Tillotson --
TP = W.MATERIAL


def test_tillotson_expanded_ideal_gas_limit():
    # far below rho0 with u >= E_cv the expanded form's exponentials vanish:
    # p = a_T rho u, and c^2 = dp/drho + p / rho^2 dp/du = a u + a^2 u
    pv = params(0.1, eos=2.0)
    a = TP["a_T"]
    rho = TP["rho0"] * np.array([0.05, 0.02])
    u = np.array([2.0, 5.0]) * TP["E_cv"]
    p, c2 = native.eos(rho, pv, u)
    assert np.allclose(p, a * rho * u, rtol=1e-15, atol=0)
    assert np.allclose(c2, a * (1 + a) * u, rtol=1e-14, atol=0)


@pytest.mark.parametrize("u", [1e6, 8e6, 3e7])
def test_tillotson_hot_compressed_value_at_reference_density(u):
    # eta = 1, chi = 0: p = (a + b / (1 + u / E0)) rho0 u, for every u (rho >= rho0 takes
    # the compressed form)
    pv = params(0.1, eos=2.0)
    r0 = TP["rho0"]
    p, _ = native.eos(np.array([r0]), pv, np.array([u]))
    want = (TP["a_T"] + TP["b_T"] / (1 + u / TP["E0_T"])) * r0 * u
    assert abs(p[0] - want) <= 1e-15 * abs(want)
