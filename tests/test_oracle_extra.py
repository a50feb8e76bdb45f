"""Pins of the energy equation (eq. energy_sph), the artificial stress of section 3.1.4
and XSPH (section 3.1.5) in the oracle, against conservation laws, the first law of
thermodynamics and two-particle closed forms (none re-types the oracle's loop)."""
import numpy as np
import pytest

import workloads as W
from oracle import native


def cube(**over):
    w = W.cube(8, 0.1, seed=31, **over)
    rng = np.random.default_rng(3)
    w.m = w.m * rng.uniform(0.8, 1.2, w.n)
    return w


def extra(w):
    return native.rhs_workload(w, want_extra=True)


def test_total_energy_conserved_pairwise():
    # d/dt sum_a m_a (v_a^2 / 2 + u_a) = 0 with viscosity, stress and unequal masses
    w = cube(alpha=1.0, beta=1.0)
    o = extra(w)
    ke = (w.m * (w.vel * o["acc"]).sum(0))
    ue = w.m * o["du"]
    scale = np.abs(ke).sum() + np.abs(ue).sum()
    assert abs(ke.sum() + ue.sum()) < 1e-12 * scale
    assert np.abs(ue).max() > 1e-3 * np.abs(ke).max()  # the energy rate is not trivially zero


def test_first_law_for_pure_pressure():
    # uniform density, no deviatoric stress, no viscosity: du = (p / rho^2) drho/dt per particle
    w = cube(alpha=0.0, beta=0.0)
    w.rho[:] = w.params["rho0"] * 1.003
    w.S[:] = 0.0
    o = extra(w)
    p = w.params["c"] ** 2 * (w.rho - w.params["rho0"])
    want = p / w.rho ** 2 * o["drho"]
    assert np.abs(o["du"] - want).max() <= 1e-12 * np.abs(want).max()


def test_viscous_heating_of_an_approaching_pair():
    w = W.two_particles((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), va=(30.0, 0.0, 0.0), vb=(-30.0, 0.0, 0.0),
                        rho=(2700.0, 2700.0), alpha=1.0, beta=1.0)
    o = extra(w)
    assert o["du"][0] > 0 and o["du"][0] == o["du"][1]
    # receding: no viscosity, and at rho0 with S = 0 no pressure work either
    w.vel = -w.vel
    assert np.all(extra(w)["du"] == 0.0)


def test_xsph_uniform_velocity_and_momentum():
    w = cube(xsph=0.5)
    w.vel[:] = np.array([[3.0], [-1.0], [2.0]])
    o = extra(w)
    assert np.array_equal(o["xv"], w.vel)
    w = cube(xsph=0.5)
    o = extra(w)
    corr = o["xv"] - w.vel
    assert np.abs((w.m * corr).sum(1)).max() < 1e-13 * np.abs(w.m * corr).sum()
    assert np.abs(corr).max() > 0


def test_xsph_two_particle_closed_form():
    h, r = 1.0, 0.4
    w = W.two_particles((0.0, 0.0, 0.0), (r, 0.0, 0.0), va=(1.0, 2.0, 0.0), vb=(-2.0, 0.5, 1.0),
                        rho=(2600.0, 2800.0), m=(1.5, 0.7), h=h, xsph=0.5)
    o = extra(w)
    Wr, _ = native.kernel(r, h)
    va, vb = w.vel[:, 0], w.vel[:, 1]
    want_a = va + 0.5 * 2 * 0.7 / (2600.0 + 2800.0) * (vb - va) * Wr
    want_b = vb + 0.5 * 2 * 1.5 / (2600.0 + 2800.0) * (va - vb) * Wr
    assert np.allclose(o["xv"][:, 0], want_a, rtol=0, atol=1e-15)
    assert np.allclose(o["xv"][:, 1], want_b, rtol=0, atol=1e-15)


def test_artificial_stress_only_in_tension():
    w = cube(eps_s=0.2)
    w.rho[:] = w.params["rho0"] * np.random.default_rng(5).uniform(1.0, 1.01, w.n)  # p >= 0
    a = extra(w)
    w.params["eps_s"] = 0.0
    b = extra(w)
    assert np.array_equal(a["acc"], b["acc"]) and np.array_equal(a["du"], b["du"])


@pytest.mark.parametrize("r_over_dmpd", [1.0, 1.5])
def test_artificial_stress_two_particle_closed_form(r_over_dmpd):
    # both particles under tension (rho < rho0), S = 0: sigma = -p I, zeta = eps_s p / rho^2 I,
    # so the extra acceleration is m_b 2 eps_s p / rho^2 (W(r) / W(dmpd))^n grad_a W: repulsive
    h, dmpd, eps_s, n_s = 1.0, 0.35, 0.2, 4.0
    r = r_over_dmpd * dmpd
    rho = 2600.0
    w = W.two_particles((0.0, 0.0, 0.0), (r, 0.0, 0.0), rho=(rho, rho), m=(1.0, 1.3), h=h,
                        alpha=0.0, eps_s=eps_s, n_s=n_s, dmpd=dmpd)
    a = extra(w)["acc"]
    w.params["eps_s"] = 0.0
    a0 = extra(w)["acc"]
    p = w.params["c"] ** 2 * (rho - w.params["rho0"])
    Wr, dWr = native.kernel(r, h)
    Wm, _ = native.kernel(dmpd, h)
    grad_a = np.array([-dWr, 0.0, 0.0])  # grad_a W = W'(r) (x_a - x_b) / r, x_a - x_b = -r e_x
    want = 1.3 * 2 * eps_s * p / rho ** 2 * (Wr / Wm) ** n_s * grad_a
    got = a[:, 0] - a0[:, 0]
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    assert got[0] < 0  # particle a sits at the origin, b at +r: pushed away from b


def test_artificial_stress_conserves_momentum():
    w = cube(eps_s=0.2)
    w.rho = w.params["rho0"] * np.random.default_rng(6).uniform(0.99, 1.01, w.n)  # mixed signs of p
    o = extra(w)
    mom = (w.m * o["acc"]).sum(1)
    assert np.abs(mom).max() < 1e-12 * np.abs(w.m * o["acc"]).sum()
    w.params["eps_s"] = 0.0
    assert np.abs(extra(w)["acc"] - o["acc"]).max() > 0  # the term acts
