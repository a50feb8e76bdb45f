"""Pins of the oracle's right-hand side against properties the paper and mathematics fix.

Each test names the passage and the property; none re-types the oracle's formulas.
  partners    section 3.5.2  lattice shell counts (integer-vector enumeration)
  density     eq. density_by_kernel_sum: lattice sum approximates int W dV = 1
  momentum    eq. accel_artvisc: pairwise antisymmetry -> total momentum conserved;
              isotropic bracket (S = 0) -> angular momentum conserved
  viscosity   section 3.1.3: only approaching pairs, repulsive, dissipative; scaling laws
  gradient    section 3.1.6: linear velocity fields reproduced up to one lattice factor
  continuity  eq. continuity_equation_sph equals -rho tr(dv/dx)
  Hooke       section 2.4: uniaxial strain rate closed form
  Jaumann     section 2.4: co-rotation of a stress in rigid rotation
  limiter     section 2.6: f_Y against the 3x3 definition of J2; idempotence
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import native

RHO0, C, MU, Y0 = 2700.0, 5000.0, 2.7e10, 3e8


def lattice(n_side=9, dx=0.1, h_over=2.4, **over):
    return W.cube(n_side, dx, seed=1, jitter=0.0, state="rest", h_over_dx=h_over, **over)


def interior(w, n_side, margin=2):
    idx = np.arange(w.n)
    ix, iy, iz = idx % n_side, (idx // n_side) % n_side, idx // (n_side * n_side)
    ok = (ix >= margin) & (ix <= n_side - 1 - margin)
    ok &= (iy >= margin) & (iy <= n_side - 1 - margin)
    ok &= (iz >= margin) & (iz <= n_side - 1 - margin)
    return idx[ok]


def run(w, **kw):
    return native.rhs_workload(w, **kw)


def test_lattice_partner_count():
    # integer vectors n != 0 with |n| < 2.4, by enumeration
    expect = sum(1 for v in itertools.product(range(-3, 4), repeat=3)
                 if v != (0, 0, 0) and v[0] ** 2 + v[1] ** 2 + v[2] ** 2 < 2.4 ** 2)
    assert expect == 56
    w = lattice(9)
    rp, col = native.neighbours(w.pos, w.h)
    cnt = np.diff(rp)
    assert np.all(cnt[interior(w, 9)] == expect)
    # partner sets are symmetric and exclude self
    pairs = set()
    for a in range(w.n):
        for b in col[rp[a]:rp[a + 1]]:
            assert b != a
            pairs.add((a, int(b)))
    assert all((b, a) in pairs for (a, b) in pairs)


def test_density_sum_is_lattice_quadrature_of_unit_integral():
    w = lattice(9)
    out = run(w)
    ratio = out["rho_sum"][interior(w, 9)] / RHO0
    # midpoint-rule quadrature of int W dV = 1 on the lattice (spacing h/2.4)
    assert np.all(np.abs(ratio - 1.0) < 2e-3)
    assert np.ptp(ratio) < 1e-12
    # the particle's own term is part of the sum (without it the sum drops by m W(0))
    assert np.all(ratio > 0.9)


def test_rest_state_is_exactly_zero():
    w = lattice(7)
    out = run(w)
    for k in ("acc", "drho", "dS", "L"):
        assert np.all(out[k] == 0.0), k


def test_uniform_velocity_is_invisible():
    w = W.config(0)
    base = run(w)
    w2 = w.copy()
    w2.vel[:] = np.array([[123.0], [-45.0], [6.5]])
    out = run(w2)
    assert np.all(out["L"] == 0.0) and np.all(out["drho"] == 0.0)
    # no viscosity for a uniform flow: acceleration is the static (pressure + stress) one
    w3 = w.copy()
    w3.vel[:] = 0.0
    assert np.array_equal(out["acc"], run(w3)["acc"])
    # Galilean invariance of the full right-hand side (to rounding)
    w4 = w.copy()
    w4.vel += np.array([[300.0], [-200.0], [100.0]])
    o4 = run(w4)
    for k in ("acc", "drho", "dS", "L"):
        assert np.abs(o4[k] - base[k]).max() <= 1e-10 * np.abs(base[k]).max(), k


def test_uniform_state_on_lattice_has_zero_interior_acceleration():
    w = lattice(9)
    w.rho[:] = 1.01 * RHO0
    w.S[:] = np.array([[1e7], [-4e6], [-6e6], [2e6], [-3e6], [5e6]])
    out = run(w)
    ii = interior(w, 9)
    scale = np.abs(out["acc"]).max()  # surface particles feel the full stress jump
    assert scale > 0
    assert np.abs(out["acc"][:, ii]).max() < 1e-12 * scale


def _rand_state(seed=3, **over):
    w = W.cube(8, 0.1, seed=seed, **over)
    rng = np.random.default_rng(seed + 100)
    w.m = w.m * rng.uniform(0.5, 1.5, size=w.n)  # unequal masses
    return w


@pytest.mark.parametrize("alpha,beta", [(0.5, 0.0), (1.0, 1.0)])
def test_linear_momentum_conserved(alpha, beta):
    w = _rand_state(alpha=alpha, beta=beta)
    out = run(w)
    ma = w.m * out["acc"]
    assert np.all(np.abs(ma.sum(1)) <= 1e-13 * np.abs(ma).sum(1))


def test_angular_momentum_conserved_without_deviatoric_stress():
    w = _rand_state(alpha=1.0, beta=1.0)
    w.S[:] = 0.0
    out = run(w)
    ma = w.m * out["acc"]
    L = np.cross(w.pos.T, ma.T)
    assert np.all(np.abs(L.sum(0)) <= 1e-13 * np.abs(L).sum(0))


def test_continuity_equals_minus_rho_trace_of_velocity_gradient():
    w = W.config(0)
    out = run(w)
    tr = out["L"][0] + out["L"][4] + out["L"][8]
    assert np.abs(out["drho"] + w.rho * tr).max() <= 1e-13 * np.abs(out["drho"]).max()


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def _mat(S6):
    xx, yy, zz, xy, xz, yz = S6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def _six(M):
    return np.stack([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def test_rotation_covariance():
    w = W.config(0)
    Q = _rot(7)
    w2 = w.copy()
    w2.pos = np.ascontiguousarray(Q @ (w.pos - 0.5) + 0.5)
    w2.vel = np.ascontiguousarray(Q @ w.vel)
    w2.S = np.ascontiguousarray(_six(np.einsum("ab,bcn,dc->adn", Q, _mat(w.S), Q)))
    a, b = run(w), run(w2)
    tol = lambda ref: 1e-10 * np.abs(ref).max()
    assert np.abs(Q @ a["acc"] - b["acc"]).max() < tol(a["acc"])
    assert np.abs(a["drho"] - b["drho"]).max() < tol(a["drho"])
    assert np.abs(a["rho_sum"] - b["rho_sum"]).max() < tol(a["rho_sum"])
    dS_rot = _six(np.einsum("ab,bcn,dc->adn", Q, _mat(a["dS"]), Q))
    assert np.abs(dS_rot - b["dS"]).max() < tol(a["dS"])
    La = a["L"].reshape(3, 3, -1)
    Lb = b["L"].reshape(3, 3, -1)
    assert np.abs(np.einsum("ab,bcn,dc->adn", Q, La, Q) - Lb).max() < tol(La)


def test_linear_velocity_field_is_reproduced():
    # section 3.1.6: for v = A x on a lattice, sum_b V_b (v_b - v_a) (x) grad W = kappa A
    # with one cubic-lattice factor kappa (1 in the continuum limit)
    w = lattice(9)
    A = np.random.default_rng(5).normal(size=(3, 3)) * 100.0
    w.vel = np.ascontiguousarray(A @ w.pos)
    out = run(w)
    ii = interior(w, 9)
    L = out["L"].reshape(3, 3, -1)[:, :, ii]
    kappa = L[0, 0, 0] / A[0, 0]
    assert abs(kappa - 1.0) < 0.05
    assert np.abs(L - kappa * A[:, :, None]).max() < 1e-10 * np.abs(A).max()


def test_simple_shear_orientation():
    # v = (g y, 0, 0): only dv_x/dy is non-zero (catches a transposed gradient)
    w = lattice(9)
    g = 50.0
    w.vel[0] = g * w.pos[1]
    out = run(w)
    ii = interior(w, 9)
    L = out["L"].reshape(3, 3, -1)[:, :, ii]
    assert np.all(L[0, 1] > 0.9 * g)
    mask = np.ones((3, 3), bool)
    mask[0, 1] = False
    assert np.abs(L[mask]).max() < 1e-10 * g


@pytest.mark.parametrize("edot", [10.0, -10.0])
def test_uniaxial_hooke_closed_form(edot):
    w = lattice(9)
    w.vel[0] = edot * w.pos[0]
    out = run(w)
    ii = interior(w, 9)
    L = out["L"].reshape(3, 3, -1)[:, :, ii]
    kappa = L[0, 0] / edot
    assert np.all(np.abs(kappa - 1.0) < 0.05) and np.ptp(kappa) < 1e-12
    dS = out["dS"][:, ii]
    ref = 2 * MU * edot * np.array([2 / 3, -1 / 3, -1 / 3])[:, None] * kappa[None, :]
    assert np.abs(dS[:3] - ref).max() < 1e-10 * np.abs(ref).max()
    assert np.abs(dS[3:]).max() < 1e-10 * np.abs(ref).max()
    assert np.allclose(dS[0] / dS[1], -2.0, rtol=1e-12)
    assert np.allclose(out["drho"][ii], -RHO0 * kappa * edot, rtol=1e-12)
    if edot > 0:  # separating pairs: no artificial viscosity, no stress, no pressure
        assert np.all(out["acc"] == 0.0)


@pytest.mark.parametrize("s", [5e7, 4e8])
def test_rigid_rotation_corotates_stress(s):
    # S(t) = Q(t) S0 Q(t)^T for v = omega z x x  =>  dS/dt = Om S0 - S0 Om,
    # with S0 = diag(s, -s, 0): dS_xy = 2 omega s (times the lattice factor and f_Y)
    w = lattice(9)
    om = 20.0
    c = w.pos.mean(1, keepdims=True)
    w.vel[0] = -om * (w.pos[1] - c[1])
    w.vel[1] = om * (w.pos[0] - c[0])
    w.S[0], w.S[1] = s, -s
    out = run(w)
    ii = interior(w, 9)
    L = out["L"].reshape(3, 3, -1)[:, :, ii]
    kappa = L[1, 0] / om
    assert np.all(np.abs(kappa - 1.0) < 0.05)
    ed = 0.5 * (L + L.transpose(1, 0, 2))
    assert np.abs(ed).max() < 1e-10 * om
    assert np.abs(out["drho"][ii]).max() < 1e-10 * RHO0 * om
    J2 = s * s  # S:S / 2 for diag(s, -s, 0)
    f = min(Y0 ** 2 / (3 * J2), 1.0)
    dS = out["dS"][:, ii]
    assert np.allclose(dS[3], 2 * kappa * om * s * f, rtol=1e-10)
    assert np.abs(dS[[0, 1, 2, 4, 5]]).max() < 1e-10 * abs(s * om)


def test_limiter_definition_and_idempotence():
    w = W.config(0)
    pre = native.prepass(w.rho, w.S, w.param_vector())
    M = _mat(w.S)
    J2 = 0.5 * np.einsum("abn,abn->n", M, M)
    f = np.minimum(Y0 ** 2 / (3 * J2), 1.0)
    assert np.allclose(pre["fy"], f, rtol=1e-14, atol=0)
    lim = (f < 1).mean()
    assert 0.05 < lim < 0.4  # both branches exercised
    pre2 = native.prepass(w.rho, w.S * pre["fy"], w.param_vector())
    assert np.all(pre2["fy"] == 1.0)
    # pressure of the linear equation of state is the isotropic part of sigma
    tr = pre["sigma"][0] + pre["sigma"][1] + pre["sigma"][2]
    assert np.allclose(-tr / 3, C * C * (w.rho - RHO0), rtol=1e-9, atol=1e-6)


def test_tension_cutoff():
    w = W.config(0)
    w.rho[:10] = 0.7 * RHO0
    pv = w.param_vector()
    pv[8] = 0.8
    pre = native.prepass(w.rho, w.S, pv)
    assert np.all(pre["p"][:10] == 0.0)
    assert np.all(pre["p"][10:] != 0.0)


# ---------------------------------------------------------------- two particles
def _pair(xb=(0.5, 0, 0), va=(0, 0, 0), vb=(0, 0, 0), rho=(RHO0, RHO0), S=None, m=(1.0, 2.0),
          **over):
    return W.two_particles((0, 0, 0), xb, va, vb, rho, S, m, h=1.0, **over)


@pytest.mark.parametrize("drho,sign", [(1.0, +1), (-1.0, -1)])
def test_pressure_repels_and_tension_attracts(drho, sign):
    w = _pair(rho=(RHO0 + drho, RHO0 + drho))
    out = run(w)
    a = out["acc"]
    rab = w.pos[:, 0] - w.pos[:, 1]
    assert sign * np.dot(a[:, 0], rab) > 0
    assert np.allclose(np.cross(a[:, 0], rab), 0.0, atol=1e-12 * np.abs(a).max())
    assert np.allclose(a[:, 1], -(w.m[0] / w.m[1]) * a[:, 0], rtol=1e-14)


def test_tensile_deviatoric_stress_along_axis_attracts():
    S = [(2e6, -1e6, -1e6, 0, 0, 0)] * 2
    out = run(_pair(S=S))
    assert out["acc"][0, 0] > 0  # a at the origin pulled towards b at +x


def test_viscosity_only_for_approaching_pairs_and_dissipative():
    app = run(_pair(va=(10.0, 0, 0), vb=(-10.0, 0, 0)))  # a at 0 moves +x towards b at 0.5
    rec = run(_pair(va=(-10.0, 0, 0), vb=(10.0, 0, 0)))
    assert np.all(rec["acc"] == 0.0)
    a = app["acc"]
    assert a[0, 0] < 0 and a[0, 1] > 0  # decelerates the approach
    m = np.array([1.0, 2.0])
    v = np.array([[10.0, -10.0], [0, 0], [0, 0]])
    assert (m * (v * a).sum(0)).sum() < 0  # kinetic energy decreases


def test_viscosity_scaling_laws():
    def visc(u, alpha, beta, rho=(RHO0, RHO0)):
        o = run(_pair(va=(u, 0, 0), vb=(-u, 0, 0), rho=rho, alpha=alpha, beta=beta))
        r = run(_pair(va=(-u, 0, 0), vb=(u, 0, 0), rho=rho, alpha=alpha, beta=beta))
        return o["acc"][0, 0] - r["acc"][0, 0]
    assert math.isclose(visc(20.0, 1.0, 0.0) / visc(10.0, 1.0, 0.0), 2.0, rel_tol=1e-13)
    assert math.isclose(visc(20.0, 0.0, 1.0) / visc(10.0, 0.0, 1.0), 4.0, rel_tol=1e-13)
    assert math.isclose(visc(10.0, 2.0, 0.0) / visc(10.0, 1.0, 0.0), 2.0, rel_tol=1e-13)
    assert visc(10.0, 0.0, 0.0) == 0.0
    # inversely proportional to the mean density of the pair
    r1 = visc(10.0, 1.0, 0.0, rho=(RHO0, RHO0))
    r2 = visc(10.0, 1.0, 0.0, rho=(1.5 * RHO0, 2.5 * RHO0))
    assert math.isclose(r1 / r2, 2.0, rel_tol=1e-13)


def test_partner_cutoff_is_strict():
    h = 1.0
    w = W.two_particles((0, 0, 0), (h, 0, 0), h=h)
    rp, col = native.neighbours(w.pos, h)
    assert rp[-1] == 0
    w = W.two_particles((0, 0, 0), (np.nextafter(h, 0), 0, 0), h=h)
    rp, col = native.neighbours(w.pos, h)
    assert rp[-1] == 2
