"""Pins of the Grady-Kipp damage model in the oracle (sections 2.7 and 3.2): the damaged
stress at d = 0, 1 and 1/2, the largest principal stress of a stress with known axes,
the activated-flaw count and growth rate of a hand-built particle, the limiter, and the
flaw distribution's Weibull law."""
import math

import numpy as np

import workloads as W
from oracle import damage, native

P = W.MATERIAL


def par(**over):
    return W.cube(4, 0.1, seed=1, **over).param_vector()


def test_zero_damage_changes_nothing():
    w = W.cube(6, 0.1, seed=2)
    a = native.rhs_workload(w)
    w.d = np.zeros(w.n)
    b = native.rhs_workload(w)
    for k in ("acc", "drho", "dS", "rho_sum"):
        assert np.array_equal(a[k], b[k]), k


def test_full_damage_takes_no_tension_and_no_deviator():
    rng = np.random.default_rng(4)
    n = 64
    rho = P["rho0"] * rng.uniform(0.97, 1.03, n)
    S = rng.normal(0.0, 1e7, (6, n))
    pre = native.prepass2(rho, S, par(), d=np.ones(n))
    p = pre["p"]
    sig = pre["sigma"]
    assert (p > 0).any() and (p < 0).any()
    assert np.all(sig[3:] == 0.0)
    for i in range(3):
        assert np.array_equal(sig[i], np.where(p >= 0, -p, 0.0))


def test_full_damage_in_tension_feels_no_force():
    w = W.cube(6, 0.1, seed=3)
    w.params.update(alpha=0.0)
    w.rho[:] = 0.98 * P["rho0"]
    w.d = np.ones(w.n)
    out = native.rhs_workload(w)
    assert np.all(out["acc"] == 0.0)


def test_half_damage_halves_tension_and_deviator_only():
    rng = np.random.default_rng(5)
    n = 64
    rho = P["rho0"] * rng.uniform(0.97, 1.03, n)
    S = rng.normal(0.0, 1e7, (6, n))
    und = native.prepass2(rho, S, par())
    half = native.prepass2(rho, S, par(), d=np.full(n, 0.5))
    p, f = und["p"], und["fy"]
    for i in range(3):
        ph = np.where(p >= 0, p, 0.5 * p)
        assert np.allclose(half["sigma"][i], 0.5 * f * S[i] - ph, rtol=1e-14, atol=1e-6)
    for i in range(3, 6):
        assert np.allclose(half["sigma"][i], 0.5 * und["sigma"][i], rtol=1e-14, atol=1e-6)


def _rotation(a, b, c):
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    Rz = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]])
    Ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    Rx = np.array([[1, 0, 0], [0, cc, -sc], [0, sc, cc]])
    return Rz @ Ry @ Rx


def test_largest_principal_stress_of_a_rotated_deviator():
    # a traceless stress with principal values (3, -1, -2) MPa on rotated axes, at rho0 so that p = 0
    Q = _rotation(0.3, -1.1, 2.0)
    T = Q @ np.diag([3e6, -1e6, -2e6]) @ Q.T
    S = np.array([[T[0, 0]], [T[1, 1]], [T[2, 2]], [T[0, 1]], [T[0, 2]], [T[1, 2]]])
    pre = native.prepass2(np.array([P["rho0"]]), S, par(Y0=1e12))
    assert pre["p"][0] == 0.0 and pre["fy"][0] == 1.0
    assert abs(damage.principal_max(pre["sigma"])[0] - 3e6) < 1e-9 * 3e6
    # a diagonal stress: the largest diagonal entry
    assert damage.principal_max(np.array([[-1.0], [4.0], [2.0], [0.0], [0.0], [0.0]]))[0] == 4.0


def test_rate_of_a_hand_built_particle():
    # uniaxial deviator diag(s, -s/2, -s/2) at rho0 (p = 0), yield far away: sigma_max = s
    s = 2.0e6
    K = P["rho0"] * P["c"] ** 2
    mu = P["mu"]
    E = 9.0 * K * mu / (3.0 * K + mu)
    eps = s / E
    S = np.array([[s], [-s / 2], [-s / 2], [0.0], [0.0], [0.0]])
    m = np.array([0.25])
    flaw_ptr = np.array([0, 3])
    flaw_eps = np.array([0.25 * eps, 0.5 * eps, 2.0 * eps])
    rate, nact, e = damage.rates(np.array([P["rho0"]]), S, m, par(Y0=1e12), flaw_ptr, flaw_eps)
    assert abs(e[0] - eps) <= 1e-14 * eps
    assert nact[0] == 2
    Rs = (3.0 * 0.25 / (4.0 * math.pi * P["rho0"])) ** (1.0 / 3.0)
    cg = 0.4 * math.sqrt((K + 4.0 / 3.0 * mu) / P["rho0"])
    assert abs(rate[0] - 2.0 * cg / Rs) <= 1e-13 * rate[0]
    # half damaged: sigma_d and (1 - d) E are both halved, so the strain is unchanged, and
    # c_g sees the weakened shear modulus; below the limiter 2/3 it still grows
    d = np.array([0.5])
    rate2, nact2, e2 = damage.rates(np.array([P["rho0"]]), S, m, par(Y0=1e12), flaw_ptr, flaw_eps, d=d)
    assert abs(e2[0] - eps) <= 1e-14 * eps and nact2[0] == 2
    cg2 = 0.4 * math.sqrt((K + 4.0 / 3.0 * 0.5 * mu) / P["rho0"])
    assert abs(rate2[0] - 2.0 * cg2 / Rs) <= 1e-13 * rate2[0]
    # at the limiter n_act / n_tot = 2/3 growth stops
    rate3, _, _ = damage.rates(np.array([P["rho0"]]), S, m, par(Y0=1e12), flaw_ptr, flaw_eps,
                               d=np.array([2.0 / 3.0 + 1e-12]))
    assert rate3[0] == 0.0
    # the reversed deviator has sigma_max = s/2: only the lowest flaw is active
    rate4, nact4, e4 = damage.rates(np.array([P["rho0"]]), -S, m, par(Y0=1e12), flaw_ptr, flaw_eps)
    assert abs(e4[0] - 0.5 * eps) <= 1e-14 * eps and nact4[0] == 1
    assert abs(rate4[0] - cg / Rs) <= 1e-13 * rate4[0]
    # isotropic compression activates nothing
    rate5, nact5, _ = damage.rates(np.array([1.01 * P["rho0"]]), 0.0 * S, m, par(), flaw_ptr, flaw_eps)
    assert rate5[0] == 0.0 and nact5[0] == 0


def test_full_damage_has_every_flaw_active_and_no_growth():
    rng = np.random.default_rng(6)
    n = 16
    ptr, eps = W.flaws(n, 1.0, 1e61, 16.0, seed=1)
    rate, nact, _ = damage.rates(P["rho0"] * np.ones(n), rng.normal(0, 1e6, (6, n)), np.ones(n),
                                 par(), ptr, eps, d=np.ones(n))
    assert np.array_equal(nact, np.diff(ptr)) and np.all(rate == 0.0)


def test_flaw_distribution_follows_the_weibull_law():
    n, V, k, m = 4096, 2.0, 1e61, 16.0
    ptr, eps = W.flaws(n, V, k, m, seed=7)
    cnt = np.diff(ptr)
    assert cnt.min() >= 1
    for a in range(0, n, 97):
        f = eps[ptr[a]:ptr[a + 1]]
        assert np.all(np.diff(f) > 0)
    total = int(ptr[-1])
    # coupon collector: mean n H_n, spread about pi n / sqrt(6)
    Hn = np.sum(1.0 / np.arange(1, n + 1))
    assert abs(total - n * Hn) < 5.0 * math.pi * n / math.sqrt(6.0)
    # flaw j has threshold (j / (k V))^(1/m): the count below eps is k V eps^m, n(eps) = k eps^m
    allf = np.sort(eps)
    j = np.arange(1, total + 1)
    assert np.allclose(allf, (j / (k * V)) ** (1.0 / m), rtol=1e-14)
    e = allf[total // 2]
    assert abs(np.sum(allf <= e) - k * V * e ** m) <= 1.0 + 1e-9 * total
