"""Pins of the Murnaghan and Tillotson equations of state (sections 2.5.2, 2.5.3) in the
oracle: reductions to the liquid equation and to the cold compression curve, the paper's
aluminium parameters, continuity across the Tillotson regions, and the sound speed
against central differences of the pressure."""
import numpy as np
import pytest

import workloads as W
from oracle import native


def par(**over):
    return W.cube(4, 0.1, seed=1, **over).param_vector()


P = W.MATERIAL


def test_murnaghan_with_unit_exponent_is_the_liquid_equation():
    rho = P["rho0"] * np.linspace(0.9, 1.1, 11)
    p1, c1 = native.eos(rho, par(eos=1.0, n_M=1.0))
    p0, c0 = native.eos(rho, par(eos=0.0))
    assert np.allclose(p1, p0, rtol=1e-13, atol=1e-13 * np.abs(p0).max())
    assert np.allclose(c1, c0, rtol=1e-15)
    w = W.cube(6, 0.1, seed=2)
    a = native.rhs_workload(w)
    w.params.update(eos=1.0, n_M=1.0)
    b = native.rhs_workload(w)
    for k in ("acc", "drho", "dS"):
        assert np.abs(a[k] - b[k]).max() <= 1e-12 * np.abs(a[k]).max(), k


def test_murnaghan_zero_pressure_and_isothermal_sound_speed():
    n = 4.0
    rho = P["rho0"] * np.linspace(0.95, 1.2, 26)
    p, c2 = native.eos(rho, par(eos=1.0, n_M=n))
    K0 = P["rho0"] * P["c"] ** 2
    assert native.eos(np.array([P["rho0"]]), par(eos=1.0, n_M=n))[0][0] == 0.0
    # closed form at eta = 1.1 and c^2 = dp/drho by central differences
    pe, _ = native.eos(np.array([1.1 * P["rho0"]]), par(eos=1.0, n_M=n))
    assert abs(pe[0] - K0 / n * (1.1 ** n - 1.0)) <= 1e-14 * abs(pe[0])
    d = 1e-4 * rho
    pp, _ = native.eos(rho + d, par(eos=1.0, n_M=n))
    pm, _ = native.eos(rho - d, par(eos=1.0, n_M=n))
    assert np.allclose((pp - pm) / (2 * d), c2, rtol=1e-7)


def test_tillotson_cold_compression_with_the_papers_aluminium():
    # u = 0, rho >= rho0: p = A chi + B chi^2 (A_T = 75.2 GPa, B_T = 65 GPa)
    eta = np.array([1.0, 1.05, 1.1, 1.3])
    p, _ = native.eos(eta * P["rho0"], par(eos=2.0))
    chi = eta - 1.0
    assert np.allclose(p, 75.2e9 * chi + 65e9 * chi ** 2, rtol=1e-14, atol=1e-3)
    assert abs(p[2] - 8.17e9) < 1e-3 * 8.17e9


def fd_sound_speed(rho, u, pv):
    dr, du = 1e-6 * rho, 1e-6 * np.maximum(u, 1e3)
    pr = (native.eos(rho + dr, pv, u)[0] - native.eos(rho - dr, pv, u)[0]) / (2 * dr)
    pu = (native.eos(rho, pv, u + du)[0] - native.eos(rho, pv, u - du)[0]) / (2 * du)
    p = native.eos(rho, pv, u)[0]
    return pr + p / rho ** 2 * pu


@pytest.mark.parametrize("eta,u", [(1.1, 1e6), (1.3, 8e6), (0.9, 1e6), (0.9, 8e6), (0.8, 2e7),
                                   (0.95, 5e6)])
def test_tillotson_sound_speed_is_the_thermodynamic_derivative(eta, u):
    pv = par(eos=2.0)
    rho = np.array([eta * P["rho0"]])
    uu = np.array([u])
    c2 = native.eos(rho, pv, uu)[1]
    want = max(fd_sound_speed(rho, uu, pv)[0], 0.0)
    assert abs(c2[0] - want) <= 1e-5 * max(abs(want), 1e5)


def test_tillotson_continuous_across_its_regions():
    pv = par(eos=2.0)
    rho = np.array([0.9 * P["rho0"]])
    for u0 in (3e6, 13.9e6):  # E_iv and E_cv in the expanded state
        lo = native.eos(rho, pv, np.array([u0 * (1 - 1e-9)]))[0][0]
        hi = native.eos(rho, pv, np.array([u0 * (1 + 1e-9)]))[0][0]
        assert abs(lo - hi) <= 1e-6 * abs(lo)
    for u0 in (5e6, 2e7):  # across rho = rho0 with vapour present
        a = native.eos(np.array([P["rho0"] * (1 + 1e-12)]), pv, np.array([u0]))[0][0]
        b = native.eos(np.array([P["rho0"] * (1 - 1e-12)]), pv, np.array([u0]))[0][0]
        assert abs(a - b) <= 1e-6 * abs(a)
    assert native.eos(np.array([P["rho0"]]), pv, np.array([0.0]))[0][0] == 0.0


def test_rhs_with_tillotson_conserves_momentum_and_uses_u():
    w = W.cube(6, 0.1, seed=3, eos=2.0)
    rng = np.random.default_rng(4)
    w.rho = P["rho0"] * rng.uniform(0.9, 1.1, w.n)
    w.u = rng.uniform(0.0, 2e7, w.n)
    o = native.rhs_workload(w)
    assert np.abs((w.m * o["acc"]).sum(1)).max() < 1e-12 * np.abs(w.m * o["acc"]).sum()
    w.u = np.zeros(w.n)
    assert np.abs(native.rhs_workload(w)["acc"] - o["acc"]).max() > 0
