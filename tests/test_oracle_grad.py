"""Pins of the gradient oracle (reverse-mode AD of the torch transcription).

  * the torch right-hand side equals the C oracle (two independent codings)
  * one right-hand side: <J^T y, u> equals central finite differences of the
    *C* oracle along random directions of every input (positions, velocities,
    density, stress) and of mu and Y0
  * leapfrog objectives: finite differences in mu, Y0 and v0 directions
  * closed forms: final momentum = initial momentum (pairwise antisymmetric
    forces) so d P / d v0_a = m_a I and d P / d(mu, Y0) = 0; with Y0 beyond any
    stress the limiter never acts and d KE / d Y0 = 0 exactly
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import autodiff as AD
from oracle import native


def small(seed=11, n_side=6, **over):
    w = W.cube(n_side, 0.1, seed=seed, **over)
    rng = np.random.default_rng(seed + 1)
    w.m = w.m * rng.uniform(0.7, 1.3, size=w.n)
    return w


def test_torch_transcription_matches_c_oracle():
    w = small(alpha=1.0, beta=1.0)
    ref = native.rhs_workload(w)
    out = AD.rhs(*AD.as_tensors(w))
    for k in ("acc", "drho", "dS", "rho_sum"):
        a, b = ref[k], out[k].numpy()
        assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max(), k
    assert np.abs(ref["L"] - out["L"].reshape(9, -1).numpy()).max() <= 1e-14 * np.abs(ref["L"]).max()


def _objective(w, y, **kw):
    o = native.rhs_workload(w, want_L=False)
    return sum(float((o[k] * y[k]).sum()) for k in y)


@pytest.mark.parametrize("which", ["pos", "vel", "rho", "S", "mu", "Y0"])
def test_rhs_vjp_matches_finite_differences(which):
    w = small(alpha=1.0, beta=1.0)
    ref = native.rhs_workload(w, want_L=False)
    rng = np.random.default_rng(5)
    y = {k: rng.normal(size=ref[k].shape) / np.abs(ref[k]).max() for k in ref}
    g = AD.rhs_vjp(w, y)
    pv = w.param_vector()
    scale = dict(pos=w.dx, vel=0.01 * 5000, rho=2700.0 * 0.01, S=6.75e7, mu=pv[3], Y0=pv[4])[which]
    if which in ("mu", "Y0"):
        u = 1.0
        ad = g[which] * u
    else:
        u = rng.normal(size=getattr(w, which).shape)
        ad = float((g[which] * u).sum())
    eps = 1e-6 * scale
    vals = []
    for sgn in (+1, -1):
        w2 = w.copy()
        if which == "mu":
            w2.params["mu"] = pv[3] + sgn * eps
        elif which == "Y0":
            w2.params["Y0"] = pv[4] + sgn * eps
        else:
            setattr(w2, which, getattr(w, which) + sgn * eps * u)
        vals.append(_objective(w2, y))
    fd = (vals[0] - vals[1]) / (2 * eps)
    assert abs(fd - ad) <= 2e-6 * max(abs(ad), 1e-300) + 1e-9, (fd, ad)


def test_leapfrog_gradients_match_finite_differences():
    w = small(seed=21, n_side=5)
    steps, dt = 4, 0.2 * w.dx / 5000.0
    g = AD.leapfrog_grad(w, steps, dt, "ke")
    pv = w.param_vector()
    for name, idx in (("mu", 3), ("Y0", 4)):
        e = 1e-6 * pv[idx]
        kw = lambda s: {name: pv[idx] + s * e}
        fd = (AD.leapfrog_value(w, steps, dt, **kw(+1)) - AD.leapfrog_value(w, steps, dt, **kw(-1))) / (2 * e)
        assert abs(fd - g[name]) <= 1e-5 * abs(g[name]), (name, fd, g[name])
    d = np.random.default_rng(3).normal(size=w.vel.shape)
    e = 1e-6 * 50.0
    fd = (AD.leapfrog_value(w, steps, dt, vel=w.vel + e * d)
          - AD.leapfrog_value(w, steps, dt, vel=w.vel - e * d)) / (2 * e)
    ad = float((g["v0"] * d).sum())
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_leapfrog_all_field_gradients_match_finite_differences():
    """Linear objective of every final field; finite differences along random
    directions of the initial positions, density and stress."""
    w = small(seed=23, n_side=5)
    steps, dt = 3, 0.2 * w.dx / 5000.0
    rng = np.random.default_rng(4)
    cot = {"pos": rng.normal(size=(3, w.n)), "vel": rng.normal(size=(3, w.n)),
           "rho": rng.normal(size=w.n) * 1e-3, "S": rng.normal(size=(6, w.n)) * 1e-9}
    g = AD.leapfrog_grad_all(w, steps, dt, cot)

    def J(**kw):
        pos, vel, rho, S, m, par = AD.as_tensors(w)
        args = dict(pos=pos, rho=rho, S=S)
        for k, v in kw.items():
            args[k] = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64))
        with torch.no_grad():
            f = AD.leapfrog(args["pos"], vel, args["rho"], args["S"], m, par, steps, dt)
        return sum(float((torch.from_numpy(cot[k]) * t).sum()) for k, t in zip(("pos", "vel", "rho", "S"), f))

    for name, base, scale in (("pos", w.pos, 1e-4 * w.dx), ("rho", w.rho, 1e-6 * 2700.0),
                              ("S", w.S, 1e-6 * 6.75e7)):
        d = rng.normal(size=base.shape)
        fd = (J(**{name: base + scale * d}) - J(**{name: base - scale * d})) / (2 * scale)
        ad = float((g[name] * d).sum())
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-300), (name, fd, ad)


@pytest.mark.parametrize("axis", ["px", "py", "pz"])
def test_momentum_objective_closed_form(axis):
    w = small(seed=31, n_side=5)
    steps, dt = 4, 0.2 * w.dx / 5000.0
    g = AD.leapfrog_grad(w, steps, dt, axis)
    k = "xyz".index(axis[1])
    expect = np.zeros_like(w.vel)
    expect[k] = w.m
    assert np.abs(g["v0"] - expect).max() <= 1e-10 * w.m.max()
    gk = AD.leapfrog_grad(w, steps, dt, "ke")
    # d P / d mu vanishes: compare with the size of the same derivative of KE / |v|
    vs = np.abs(w.vel).max()
    assert abs(g["mu"]) * vs <= 1e-8 * abs(gk["mu"])
    assert abs(g["Y0"]) * vs <= 1e-8 * abs(gk["Y0"])


def test_vjp_of_a_local_cotangent_is_local():
    """A cotangent supported within 0.7 h of a point gives gradients that vanish beyond
    1.7 h, and the product over the particles within 2.75 h alone equals the whole set's
    there (every particle it involves has all its partners in that ball): the premise of
    the full-size adjoint comparison on the GPU."""
    w = W.config(0)
    c = 2000
    sup = native.ball(w.pos, w.pos[:, c], 0.7 * w.h)
    sub = native.ball(w.pos, w.pos[:, c], 2.75 * w.h)
    fwd = native.rhs(w.pos, w.vel, w.rho, w.S, w.m, w.param_vector(), targets=sup)
    rng = np.random.default_rng(1)
    cot = {"acc": np.zeros((3, w.n)), "drho": np.zeros(w.n), "dS": np.zeros((6, w.n)),
           "rho_sum": np.zeros(w.n)}
    for k in cot:
        cot[k][..., sup] = rng.normal(size=cot[k][..., sup].shape) / np.abs(fwd[k]).max()
    full = AD.rhs_vjp(w, cot)
    loc = AD.rhs_vjp(w.take(sub), {k: np.ascontiguousarray(v[..., sub]) for k, v in cot.items()})
    near = native.ball(w.pos, w.pos[:, c], 1.7 * w.h)
    far = np.ones(w.n, dtype=bool)
    far[near] = False
    assert len(sup) > 5 and len(sub) < w.n // 4
    for k in ("pos", "vel", "rho", "S"):
        assert np.array_equal(full[k][..., sub], loc[k]), k
        assert not np.any(full[k][..., far]), k
        assert np.any(full[k]), k
    for k in ("mu", "Y0"):  # sums over the particles, in another order
        assert abs(full[k] - loc[k]) <= 1e-14 * abs(full[k]), k


def test_unlimited_yield_stress_has_zero_gradient():
    w = small(seed=41, n_side=5, Y0=1e30)
    g = AD.leapfrog_grad(w, 3, 0.2 * w.dx / 5000.0, "ke")
    assert g["Y0"] == 0.0
    assert g["mu"] != 0.0


def test_torch_transcription_with_damage_matches_c_oracle_and_finite_differences():
    # a fixed damage field (section 2.7): the transcription against the C oracle, and its
    # reverse-mode product against central differences of the C oracle in rho and S
    w = small(seed=13, alpha=1.0, beta=1.0)
    rng = np.random.default_rng(14)
    w.d = rng.uniform(0.0, 1.0, w.n)
    w.rho = w.params["rho0"] * rng.uniform(0.995, 1.005, w.n)  # both signs of p
    ref = native.rhs_workload(w)
    out = AD.rhs(*AD.as_tensors(w), d=w.d)
    for k in ("acc", "drho", "dS", "rho_sum"):
        a, b = ref[k], out[k].numpy()
        assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max(), k
    y = {k: rng.normal(size=ref[k].shape) / np.abs(ref[k]).max() for k in ("acc", "drho", "dS", "rho_sum")}
    g = AD.rhs_vjp(w, y)
    for which, scale in (("rho", 2700.0 * 1e-4), ("S", 6.75e7)):
        u = rng.normal(size=getattr(w, which).shape)
        ad = float((g[which] * u).sum())
        eps = 1e-6 * scale
        vals = []
        for sgn in (+1, -1):
            wp = w.copy()
            wp.d = w.d
            setattr(wp, which, getattr(w, which) + sgn * eps * u)
            vals.append(_objective(wp, y))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (which, fd, ad)


@pytest.mark.parametrize("rho_cut", [0.0, 0.999])
def test_torch_transcription_with_murnaghan_matches_c_oracle_and_finite_differences(rho_cut):
    # the Murnaghan equation (section 2.5.2) with its per-particle sound speed in Pi
    w = small(seed=15, alpha=1.0, beta=1.0, eos=1.0, n_M=4.0, rho_cut=rho_cut)
    rng = np.random.default_rng(16)
    w.rho = w.params["rho0"] * rng.uniform(0.97, 1.03, w.n)
    ref = native.rhs_workload(w)
    out = AD.rhs(*AD.as_tensors(w))
    for k in ("acc", "drho", "dS", "rho_sum"):
        a, b = ref[k], out[k].numpy()
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), k
    y = {k: rng.normal(size=ref[k].shape) / np.abs(ref[k]).max() for k in ("acc", "drho", "dS", "rho_sum")}
    g = AD.rhs_vjp(w, y)
    u = rng.normal(size=w.n)
    ad = float((g["rho"] * u).sum())
    eps = 1e-7 * 2700.0
    vals = []
    for sgn in (+1, -1):
        wp = w.copy()
        wp.rho = w.rho + sgn * eps * u
        vals.append(_objective(wp, y))
    fd = (vals[0] - vals[1]) / (2 * eps)
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    # the sound speed's dependence on rho matters: the liquid transcription differs
    w.params["eos"] = 0.0
    assert np.abs(AD.rhs(*AD.as_tensors(w))["acc"].numpy() - ref["acc"]).max() > 1e-3 * np.abs(ref["acc"]).max()


@pytest.mark.parametrize("n_s", [4.0, 2.5])
def test_torch_transcription_with_artificial_stress_matches_c_oracle_and_finite_differences(n_s):
    # the artificial stress (section 3.1.4), half the particles in tension
    w = small(seed=17, alpha=1.0, beta=1.0, eps_s=0.2, n_s=n_s)
    rng = np.random.default_rng(18)
    w.rho = w.params["rho0"] * rng.uniform(0.99, 1.01, w.n)
    ref = native.rhs_workload(w)
    out = AD.rhs(*AD.as_tensors(w))
    for k in ("acc", "drho", "dS", "rho_sum"):
        a, b = ref[k], out[k].numpy()
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), k
    y = {k: rng.normal(size=ref[k].shape) / np.abs(ref[k]).max() for k in ("acc", "drho", "dS", "rho_sum")}
    g = AD.rhs_vjp(w, y)
    for which, scale in (("pos", w.dx), ("S", 6.75e7), ("rho", 2700.0 * 1e-4)):
        u = rng.normal(size=getattr(w, which).shape)
        ad = float((g[which] * u).sum())
        eps = 1e-6 * scale
        vals = []
        for sgn in (+1, -1):
            wp = w.copy()
            setattr(wp, which, getattr(w, which) + sgn * eps * u)
            vals.append(_objective(wp, y))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (which, fd, ad)
    w.params["eps_s"] = 0.0  # the artificial stress acts on this state
    assert np.abs(AD.rhs(*AD.as_tensors(w))["acc"].numpy() - ref["acc"]).max() > 1e-6 * np.abs(ref["acc"]).max()


def test_torch_transcription_energy_and_xsph_match_c_oracle_and_finite_differences():
    # du/dt (section 3.1.2) and dx/dt with XSPH (section 3.1.5), with the artificial
    # stress on (excluded from the energy bracket) and the Murnaghan sound speeds
    w = small(seed=19, alpha=1.0, beta=1.0, eps_s=0.2, n_s=4.0, xsph=0.5, eos=1.0, n_M=4.0)
    rng = np.random.default_rng(20)
    w.rho = w.params["rho0"] * rng.uniform(0.99, 1.01, w.n)
    ref = native.rhs_workload(w, want_extra=True)
    out = AD.rhs(*AD.as_tensors(w))
    for k in ("du", "xv"):
        a, b = ref[k], out[k].detach().numpy()
        if k == "xv":
            a, b = a - w.vel, b - w.vel  # the XSPH correction itself
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), k
    y = {"du": rng.normal(size=w.n) / np.abs(ref["du"]).max(),
         "xv": rng.normal(size=(3, w.n)) / np.abs(ref["xv"] - w.vel).max()}
    g = AD.rhs_vjp(w, y)

    def obj(wp):
        o = native.rhs_workload(wp, want_extra=True)
        return float((o["du"] * y["du"]).sum() + (o["xv"] * y["xv"]).sum())

    for which, scale in (("pos", w.dx), ("vel", 50.0), ("rho", 2700.0 * 1e-4), ("S", 6.75e7)):
        u = rng.normal(size=getattr(w, which).shape)
        ad = float((g[which] * u).sum())
        eps = 1e-6 * scale
        vals = []
        for sgn in (+1, -1):
            wp = w.copy()
            setattr(wp, which, getattr(w, which) + sgn * eps * u)
            vals.append(obj(wp))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (which, fd, ad)


@pytest.mark.parametrize("regime", ["compressed", "expanded", "band", "mixed"])
def test_torch_transcription_with_tillotson_matches_c_oracle_and_finite_differences(regime):
    # the Tillotson equation (section 2.5.3) in each of its regions: the sound speed
    # comes from autograd here and from hand-derived partials in the C oracle, and
    # the gradient reaches u through the pressure and through the sound speed
    w = small(seed=19, alpha=1.0, beta=1.0, eos=2.0)
    rng = np.random.default_rng(20)
    rho0, Eiv, Ecv = w.params["rho0"], w.params["E_iv"], w.params["E_cv"]
    lo, hi = {"compressed": (1.001, 1.03), "expanded": (0.97, 0.999), "band": (0.97, 0.999),
              "mixed": (0.97, 1.03)}[regime]
    w.rho = rho0 * rng.uniform(lo, hi, w.n)
    if regime == "compressed":
        w.u = rng.uniform(0.0, 2e7, w.n)
    elif regime == "expanded":
        w.u = rng.uniform(1.05 * Ecv, 1.5 * Ecv, w.n)
    elif regime == "band":
        w.u = rng.uniform(1.05 * Eiv, 0.95 * Ecv, w.n)
    else:
        w.u = rng.choice([0.5 * Eiv, 0.5 * (Eiv + Ecv), 1.3 * Ecv], w.n) * rng.uniform(0.95, 1.05, w.n)
    ref = native.rhs_workload(w, want_L=False, want_extra=True)
    pos, vel, rho, S, m, par = AD.as_tensors(w)
    out = AD.rhs(pos, vel, rho, S, m, par, u=torch.from_numpy(w.u))
    for k in ("acc", "drho", "dS", "rho_sum", "du"):
        a, b = ref[k], out[k].detach().numpy()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), k
    keys = ("acc", "drho", "dS", "rho_sum", "du")
    y = {k: rng.normal(size=ref[k].shape) / np.abs(ref[k]).max() for k in keys}
    g = AD.rhs_vjp(w, y)

    def objective(wp):
        o = native.rhs_workload(wp, want_L=False, want_extra=True)
        return sum(float((o[k] * y[k]).sum()) for k in keys)

    for field, scale in (("rho", 1e-7 * rho0), ("u", 1e-7 * Ecv)):
        dirn = rng.normal(size=w.n)
        ad = float((g[field] * dirn).sum())
        vals = []
        for sgn in (+1, -1):
            wp = w.copy()
            setattr(wp, field, getattr(w, field) + sgn * scale * dirn)
            vals.append(objective(wp))
        fd = (vals[0] - vals[1]) / (2 * scale)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (field, fd, ad)
    # u acts through the pressure and the sound speed: its gradient is not zero
    assert np.abs(g["u"]).max() > 0.0
