"""GPU parity of the adjoint path: sph_rhs_adjoint against reverse-mode AD of the
oracle, the leapfrog and its reverse sweep against the oracle's trajectory and
gradients, and, at the full 64,000-particle / 20-step size, central finite
differences and the momentum closed form (properties that hold at any size)."""
import ctypes as C
import numpy as np
import pytest
import torch

import workloads as W
from oracle import autodiff as AD
from oracle import native
import paper_1604_03290_amd as P
from paper_1604_03290_amd import _lib as L

pytestmark = pytest.mark.gpu


def gpu_state(w):
    return P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    s = np.abs(b).max()
    return np.abs(a - b).max() / s if s > 0 else np.abs(a - b).max()


def small(name):
    if name == "cube10":
        return W.cube(10, 0.1, seed=21)
    if name == "cube8_visc":
        w = W.cube(8, 0.1, seed=22, alpha=1.0, beta=1.0, rho_cut=0.99)
        w.m = w.m * np.random.default_rng(2).uniform(0.8, 1.2, w.n)
        return w
    if name == "cube16":
        return W.config(0)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["cube10", "cube8_visc", "cube16"])
@pytest.mark.parametrize("pairs", [False, True])
def test_rhs_adjoint_matches_oracle(name, pairs):
    w = small(name)
    ref_out = native.rhs_workload(w, want_L=False)
    rng = np.random.default_rng(7)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ref_out}
    ref = AD.rhs_vjp(w, cot)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=pairs)
    cg = {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()}
    got = P.sph_rhs_adjoint(g, st, w.params, cg)
    assert P.workspace_status(got["_ws"]) == 0
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    assert abs(float(got["Y0"]) - ref["Y0"]) <= 1e-11 * abs(ref["Y0"])
    # bit-for-bit reproducible
    again = P.sph_rhs_adjoint(g, st, w.params, cg)
    for k in ("pos", "vel", "rho", "S", "mu", "Y0"):
        assert torch.equal(got[k], again[k]), k


@pytest.mark.parametrize("name", ["cube10", "cube8_visc"])
@pytest.mark.parametrize("pairs", [False, True])
def test_rhs_adjoint_corrected_matches_oracle(name, pairs):
    """The correction tensor of section 3.1.6 in the adjoint: the cotangent of the
    moment matrix and its pair terms, against reverse-mode AD of the oracle."""
    w = small(name)
    w.params["correction"] = 1.0
    ref_out = native.rhs_workload(w, want_L=False)
    rng = np.random.default_rng(17)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ref_out}
    ref = AD.rhs_vjp(w, cot)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=pairs)
    cg = {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()}
    got = P.sph_rhs_adjoint(g, st, w.params, cg)
    assert P.workspace_status(got["_ws"]) == 0
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    assert abs(float(got["Y0"]) - ref["Y0"]) <= 1e-11 * abs(ref["Y0"])
    # the comparison has teeth: the uncorrected gradient differs
    w.params["correction"] = 0.0
    plain = AD.rhs_vjp(w, cot)
    assert rel(plain["pos"], ref["pos"]) > 1e-4


def test_rhs_adjoint_partial_cotangents():
    w = small("cube10")
    ref_out = native.rhs_workload(w, want_L=False)
    rng = np.random.default_rng(8)
    cot = {"rho_sum": rng.normal(size=w.n)}
    full = {k: np.zeros_like(v) for k, v in ref_out.items()}
    full.update(cot)
    ref = AD.rhs_vjp(w, full)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h)
    got = P.sph_rhs_adjoint(g, st, w.params, {"rho_sum": torch.as_tensor(cot["rho_sum"]).cuda()})
    assert rel(got["pos"].cpu().numpy(), ref["pos"]) < 1e-11
    assert float(got["mu"]) == 0.0 and np.all(got["vel"].cpu().numpy() == 0.0)


def run_leapfrog(w, steps, skin_dx=0.5, pairs=True, cells_per_h=1):
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=skin_dx * w.dx, cells_per_h=cells_per_h, pairs=pairs)
    fin, ck = P.sph_leapfrog(g, st, w.params, w.dt, steps)
    assert P.workspace_status(fin._ws) == 0
    return st, g, fin, ck


def test_leapfrog_matches_oracle_trajectory():
    w = small("cube10")
    steps = 6
    _, _, fin, _ = run_leapfrog(w, steps)
    pos, vel, rho, S, m, par = AD.as_tensors(w)
    with torch.no_grad():
        x, v, r, s = AD.leapfrog(pos, vel, rho, S, m, par, steps, w.dt)
    assert rel(fin.pos.cpu().numpy() - w.pos, x.numpy() - w.pos) < 1e-11
    assert rel(fin.vel.cpu().numpy(), v.numpy()) < 1e-11
    assert rel(fin.rho.cpu().numpy() - w.rho, r.numpy() - w.rho) < 1e-10
    assert rel(fin.S.cpu().numpy(), s.numpy()) < 1e-11


@pytest.mark.parametrize("name,steps,pairs,cph", [("cube10", 8, False, 1), ("cube10", 8, True, 1),
                                                  ("cube10", 8, True, 2), ("cube8_visc", 20, True, 1)])
def test_leapfrog_gradient_matches_oracle(name, steps, pairs, cph):
    w = small(name)
    st, g, fin, ck = run_leapfrog(w, steps, pairs=pairs, cells_per_h=cph)
    cot = {"vel": (fin.vel * fin.m).contiguous()}  # d KE / d v_final
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, steps, ck, cot)
    assert P.workspace_status(got["_ws"]) == 0
    ref = AD.leapfrog_grad(w, steps, w.dt, "ke")
    assert rel(got["vel"].cpu().numpy(), ref["v0"]) < 1e-10
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-10 * abs(ref["mu"])
    assert abs(float(got["Y0"]) - ref["Y0"]) <= 1e-10 * abs(ref["Y0"])


def test_leapfrog_gradient_all_fields_matches_oracle():
    """A linear objective of every final field: gradients of every initial field
    (exercises the slot-order permutations of state, cotangent and gradient)."""
    w = small("cube8_visc")
    steps = 6
    st, g, fin, ck = run_leapfrog(w, steps, pairs=True, cells_per_h=2)
    rng = np.random.default_rng(11)
    cot = {"pos": rng.normal(size=(3, w.n)), "vel": rng.normal(size=(3, w.n)),
           "rho": rng.normal(size=w.n) * 1e-3, "S": rng.normal(size=(6, w.n)) * 1e-9}
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, steps, ck,
                                 {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()})
    assert P.workspace_status(got["_ws"]) == 0
    ref = AD.leapfrog_grad_all(w, steps, w.dt, cot)
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-10, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-10 * abs(ref["mu"])
    assert abs(float(got["Y0"]) - ref["Y0"]) <= 1e-10 * abs(ref["Y0"])
    # the final state itself
    pos, vel, rho, S, m, par = AD.as_tensors(w)
    with torch.no_grad():
        x, v, r, s = AD.leapfrog(pos, vel, rho, S, m, par, steps, w.dt)
    assert rel(fin.pos.cpu().numpy() - w.pos, x.numpy() - w.pos) < 1e-11
    assert rel(fin.S.cpu().numpy(), s.numpy()) < 1e-11


# ------------------------------------------------ full size: 64,000 particles, 20 steps
@pytest.fixture(scope="module")
def cube40():
    w = W.config(3)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.5 * w.dx, pairs=True)
    return w, st, g


def _ke(w, st, g, params=None, vel=None):
    s = st if vel is None else P.ParticleState(st.pos, vel, st.rho, st.S, st.m)
    fin, _ = P.sph_leapfrog(g, s, params or w.params, w.dt, w.steps, checkpoints=False)
    assert P.workspace_status(fin._ws) == 0
    return 0.5 * float((fin.m * (fin.vel * fin.vel).sum(0)).sum())


def test_full_size_gradient_matches_finite_differences(cube40):
    w, st, g = cube40
    fin, ck = P.sph_leapfrog(g, st, w.params, w.dt, w.steps)
    assert P.workspace_status(fin._ws) == 0
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, w.steps, ck, {"vel": (fin.vel * fin.m).contiguous()})
    for name in ("mu", "Y0"):
        e = 1e-6 * w.params[name]
        pp = dict(w.params, **{name: w.params[name] + e})
        pm = dict(w.params, **{name: w.params[name] - e})
        fd = (_ke(w, st, g, pp) - _ke(w, st, g, pm)) / (2 * e)
        ad = float(got[name])
        assert abs(fd - ad) <= 1e-5 * abs(ad), (name, fd, ad)

# The artificial-viscosity switch (Pi only for approaching pairs) and the limiter's min()
# have derivative jumps; central differences along velocity directions cross many of
# them over 20 steps.  On the same full-size launch with both switched off (alpha = 0,
# Y0 beyond any stress) the objective is smooth and the check is tight.
def test_full_size_velocity_gradient_matches_finite_differences(cube40):
    w, st, g = cube40
    pr = dict(w.params, alpha=0.0, Y0=1e30)
    fin, ck = P.sph_leapfrog(g, st, pr, w.dt, w.steps)
    got = P.sph_leapfrog_adjoint(g, st, pr, w.dt, w.steps, ck, {"vel": (fin.vel * fin.m).contiguous()})
    assert float(got["Y0"]) == 0.0
    d = torch.as_tensor(np.random.default_rng(3).normal(size=w.vel.shape)).cuda()
    e = 1e-4 * 50.0  # rounding of KE (~1e8) over 2e * |dJ| stays near 1e-8
    fd = (_ke(w, st, g, pr, vel=(st.vel + e * d).contiguous())
          - _ke(w, st, g, pr, vel=(st.vel - e * d).contiguous())) / (2 * e)
    ad = float((got["vel"] * d).sum())
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    e = 1e-6 * w.params["mu"]
    fd = (_ke(w, st, g, dict(pr, mu=pr["mu"] + e)) - _ke(w, st, g, dict(pr, mu=pr["mu"] - e))) / (2 * e)
    assert abs(fd - float(got["mu"])) <= 1e-6 * abs(float(got["mu"]))


def test_full_size_momentum_gradient_closed_form(cube40):
    w, st, g = cube40
    fin, ck = P.sph_leapfrog(g, st, w.params, w.dt, w.steps)
    cot = torch.zeros_like(fin.vel)
    cot[0] = fin.m  # J = sum_a m_a v_a^x
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, w.steps, ck, {"vel": cot})
    gv = got["vel"].cpu().numpy()
    m = w.m
    assert np.abs(gv[0] - m).max() <= 1e-9 * m.max()
    assert np.abs(gv[1:]).max() <= 1e-9 * m.max()
    # momentum does not depend on mu or Y0: compare with the kinetic-energy sensitivity
    ke = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, w.steps, ck, {"vel": (fin.vel * fin.m).contiguous()})
    vs = float(torch.abs(st.vel).max())
    assert abs(float(got["mu"])) * vs <= 1e-8 * abs(float(ke["mu"]))
    assert abs(float(got["Y0"])) * vs <= 1e-8 * abs(float(ke["Y0"]))


def test_full_size_gradient_matches_oracle_golden(cube40):
    """The oracle's gradient of the same 64,000-particle, 20-step trajectory, written by
    tests/golden/make_cube40_gradient.py (oracle only)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cube40_gradient.json")))
    w, st, g = cube40
    assert gold["n"] == w.n and gold["steps"] == w.steps and abs(gold["dt"] - w.dt) < 1e-20
    fin, ck = P.sph_leapfrog(g, st, w.params, w.dt, w.steps)
    J = 0.5 * float((fin.m * (fin.vel * fin.vel).sum(0)).sum())
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, w.steps, ck, {"vel": (fin.vel * fin.m).contiguous()})
    assert abs(J - gold["J"]) <= 1e-12 * abs(gold["J"])
    assert abs(float(got["mu"]) - gold["mu"]) <= 1e-9 * abs(gold["mu"])
    assert abs(float(got["Y0"]) - gold["Y0"]) <= 1e-9 * abs(gold["Y0"])
    d = np.random.default_rng(gold["direction_seed"]).normal(size=w.vel.shape)
    gv = got["vel"].cpu().numpy()
    assert abs(float((gv * d).sum()) - gold["v0_dot_direction"]) <= 1e-9 * abs(gold["v0_dot_direction"])
    ref = np.array(gold["v0_sample"])
    assert np.abs(gv[:, gold["sample_index"]] - ref).max() <= 1e-9 * np.abs(ref).max()


def test_leapfrog_gradient_corrected_matches_oracle():
    """Leapfrog and reverse sweep with the correction tensor: every field's gradient
    (the checkpoint carries the moment matrix beside L)."""
    w = small("cube8_visc")
    w.params["correction"] = 1.0
    steps = 6
    st, g, fin, ck = run_leapfrog(w, steps, pairs=True, cells_per_h=2)
    rng = np.random.default_rng(12)
    cot = {"pos": rng.normal(size=(3, w.n)), "vel": rng.normal(size=(3, w.n)),
           "rho": rng.normal(size=w.n) * 1e-3, "S": rng.normal(size=(6, w.n)) * 1e-9}
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, steps, ck,
                                 {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()})
    assert P.workspace_status(got["_ws"]) == 0
    ref = AD.leapfrog_grad_all(w, steps, w.dt, cot)
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-10, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-10 * abs(ref["mu"])
    assert abs(float(got["Y0"]) - ref["Y0"]) <= 1e-10 * abs(ref["Y0"])
    pos, vel, rho, S, m, par = AD.as_tensors(w)
    with torch.no_grad():
        x, v, r, s = AD.leapfrog(pos, vel, rho, S, m, par, steps, w.dt)
    assert rel(fin.pos.cpu().numpy() - w.pos, x.numpy() - w.pos) < 1e-11
    assert rel(fin.S.cpu().numpy(), s.numpy()) < 1e-11


def test_nonuniform_adjoint_matches_directional_derivative():
    """At 8,388,608 particles (9 to 255 partners): <adjoint, direction> equals the
    central difference of <cotangent, sph_rhs> along a direction that moves the
    densities and stresses at random and the velocities by a small rigid rotation (a
    property that holds at any size).  The rotation leaves every w = (v_a - v_b).r
    unchanged, so no pair crosses the viscosity switch w = 0 and the difference is
    free of kinks; the viscosity's velocity derivative is pinned at smaller sizes."""
    w = W.config(4)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.1 * w.dx, cells_per_h=2, pairs=True)
    n = w.n
    gen = torch.Generator("cuda").manual_seed(3)
    cot = {"acc": torch.randn(3, n, dtype=torch.float64, device="cuda", generator=gen),
           "drho": torch.randn(n, dtype=torch.float64, device="cuda", generator=gen),
           "dS": torch.randn(6, n, dtype=torch.float64, device="cuda", generator=gen)}
    base = P.sph_rhs(g, st, w.params)
    for k in cot:  # comparable weight for every output
        cot[k] /= base[k].abs().max()
    grad = P.sph_rhs_adjoint(g, st, w.params, cot)
    assert P.workspace_status(grad["_ws"]) == 0
    eps = 1e-7
    om = torch.randn(3, dtype=torch.float64, device="cuda", generator=gen)
    om *= eps * float(st.vel.abs().max()) / float((st.pos - st.pos.mean(1, keepdim=True)).abs().max())
    xc = st.pos - st.pos.mean(1, keepdim=True)
    dv = torch.stack([om[1] * xc[2] - om[2] * xc[1], om[2] * xc[0] - om[0] * xc[2],
                      om[0] * xc[1] - om[1] * xc[0]])
    dr = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen) * eps * float(st.rho.mean())
    dS = torch.randn(6, n, dtype=torch.float64, device="cuda", generator=gen) * eps * float(st.S.abs().max())
    pred = float((grad["vel"] * dv).sum() + (grad["rho"] * dr).sum() + (grad["S"] * dS).sum())

    def outputs(sign):
        s2 = P.ParticleState(st.pos, (st.vel + sign * dv).contiguous(), (st.rho + sign * dr).contiguous(),
                             (st.S + sign * dS).contiguous(), st.m)
        return P.sph_rhs(g, s2, w.params)

    op, om_ = outputs(1.0), outputs(-1.0)
    # difference the outputs element by element before the weighted sum (no cancellation
    # between two large totals)
    fd = sum(float((cot[k] * (op[k] - om_[k])).sum()) for k in cot) / 2.0
    assert abs(fd - pred) <= 1e-6 * abs(pred), (fd, pred)


@pytest.mark.parametrize("corr", [False, True])
@pytest.mark.parametrize("pairs", [False, True])
def test_rhs_adjoint_reuses_the_forward_velocity_gradient(corr, pairs):
    """sph_rhs's vgrad output handed to sph_rhs_adjoint: the same gradients as the
    adjoint that forms the velocity gradient itself (to rounding: the two kernels sum
    the same terms), both against the oracle's reverse-mode product."""
    w = small("cube8_visc")
    w.params["correction"] = 1.0 if corr else 0.0
    ref_out = native.rhs_workload(w, want_L=False)
    rng = np.random.default_rng(27)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ref_out}
    ref = AD.rhs_vjp(w, cot)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=pairs)
    fwd = P.sph_rhs(g, st, w.params, "fp64", vgrad=True)
    assert fwd["vgrad"].shape == (w.n, 15 if corr else 9)
    if not corr:  # row s is slot s's L, row by row: the oracle's L of user perm[s]
        Lu = np.empty((9, w.n))
        Lu[:, g.perm.cpu().numpy()] = fwd["vgrad"].cpu().numpy().T
        assert rel(Lu, native.rhs_workload(w)["L"]) < 1e-12
    plain = P.sph_rhs(g, st, w.params, "fp64")
    for k in ("acc", "drho", "dS", "rho_sum"):  # writing vgrad changes no output
        assert torch.equal(fwd[k], plain[k]), k
    cg = {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()}
    own = P.sph_rhs_adjoint(g, st, w.params, cg)
    got = P.sph_rhs_adjoint(g, st, w.params, cg, vgrad=fwd["vgrad"])
    assert P.workspace_status(got["_ws"]) == 0
    # the forward's operand records handed over as well: the same records, so the same
    # gradients bit for bit (also with the records alone)
    fr = P.sph_rhs(g, st, w.params, "fp64", vgrad=True, records=True)
    assert fr["rec"].shape == (w.n, 16) and torch.equal(fr["vgrad"], fwd["vgrad"])
    both = P.sph_rhs_adjoint(g, st, w.params, cg, vgrad=fr["vgrad"], rec=fr["rec"])
    recs = P.sph_rhs_adjoint(g, st, w.params, cg, rec=fr["rec"])
    # the FP32-compensated form writes the same FP64 records
    f32 = P.sph_rhs(g, st, w.params, "fp32comp", records=True)
    assert torch.equal(f32["rec"], fr["rec"])
    for k in ("pos", "vel", "rho", "S", "mu", "Y0"):
        assert torch.equal(both[k], got[k]), k
        assert torch.equal(recs[k], own[k]), k
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), own[k].cpu().numpy()) < 1e-13, k
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k
    for k in ("mu", "Y0"):
        assert abs(float(got[k]) - ref[k]) <= 1e-11 * abs(ref[k]), k
    # the FP32-compensated form does not write it
    with pytest.raises(L.SphError):
        P.sph_rhs(g, st, w.params, "fp32comp", vgrad=True)


def test_nonuniform_adjoint_local_cotangent_matches_oracle():
    """At 8,388,608 particles, sph_rhs_adjoint against the oracle's reverse-mode product,
    element by element.  The cotangent is random on the particles within 0.7 h of a
    centre and zero elsewhere (one centre in each body: the dense sphere, the sphere and
    the sparse shell).  Every term of the product then involves only particles within
    2 h of that support (a gradient reaches the partners of the support, and the
    velocity gradients of the support need their partners), so the oracle's product
    over the particles within 2.75 h of the centre is the exact value there, and the
    GPU's gradient must vanish exactly everywhere else."""
    w = W.config(4)
    idx = W.subsample(w.n, 512, seed=31)
    deg = np.diff(native.neighbours(w.pos, w.h, idx)[0])
    centres = [idx[np.argmax(deg)], idx[np.argmin(np.abs(deg - 60))], idx[np.argmin(deg)]]
    assert deg.max() > 200 and deg.min() < 30
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.1 * w.dx, cells_per_h=2, pairs=True)
    rng = np.random.default_rng(32)
    for c in centres:
        sup = native.ball(w.pos, w.pos[:, c], 0.7 * w.h)
        sub = native.ball(w.pos, w.pos[:, c], 2.75 * w.h)
        fwd = native.rhs(w.pos, w.vel, w.rho, w.S, w.m, w.param_vector(), targets=sup)
        cot = {"acc": np.zeros((3, w.n)), "drho": np.zeros(w.n), "dS": np.zeros((6, w.n)),
               "rho_sum": np.zeros(w.n)}
        for k in cot:  # comparable weight for every output
            cot[k][..., sup] = rng.normal(size=cot[k][..., sup].shape) / np.abs(fwd[k]).max()
        got = P.sph_rhs_adjoint(g, st, w.params,
                                {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()})
        assert P.workspace_status(got["_ws"]) == 0
        ref = AD.rhs_vjp(w.take(sub), {k: np.ascontiguousarray(v[..., sub]) for k, v in cot.items()})
        out = np.ones(w.n, dtype=bool)
        out[sub] = False
        for k in ("pos", "vel", "rho", "S"):
            gk = got[k].cpu().numpy()
            assert rel(gk[..., sub], ref[k]) < 1e-11, (int(c), k, rel(gk[..., sub], ref[k]))
            assert not np.any(gk[..., out]), (int(c), k)
        assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"]), int(c)
        assert abs(float(got["Y0"]) - ref["Y0"]) <= 1e-11 * max(abs(ref["Y0"]), 1e-300), int(c)


def test_autograd_function_matches_adjoint_and_oracle():
    # SphRhs: forward = sph_rhs, backward = sph_rhs_adjoint, through torch.autograd
    w = small("cube8_visc")
    ref_out = native.rhs_workload(w, want_L=False)
    rng = np.random.default_rng(9)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ref_out}
    ref = AD.rhs_vjp(w, cot)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=True)
    leaves = [t.clone().requires_grad_(True) for t in (st.pos, st.vel, st.rho, st.S)]
    mu = torch.tensor(w.params["mu"], dtype=torch.float64, device="cuda", requires_grad=True)
    Y0 = torch.tensor(w.params["Y0"], dtype=torch.float64, device="cuda", requires_grad=True)
    outs = P.SphRhs.apply(*leaves, mu, Y0, g, w.params, st.m)
    direct = P.sph_rhs(g, st, w.params, "fp64", vgrad=True)
    for k, o in zip(("acc", "drho", "dS", "rho_sum"), outs):
        assert torch.equal(o, direct[k]), k
    loss = sum((o * torch.as_tensor(cot[k]).cuda()).sum()
               for k, o in zip(("acc", "drho", "dS", "rho_sum"), outs))
    loss.backward()
    cg = {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()}
    # the backward reuses the forward's velocity gradient
    adj = P.sph_rhs_adjoint(g, st, w.params, cg, vgrad=direct["vgrad"])
    for k, t in zip(("pos", "vel", "rho", "S"), leaves):
        assert torch.equal(t.grad, adj[k]), k
        assert rel(t.grad.cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(mu.grad) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    assert abs(float(Y0.grad) - ref["Y0"]) <= 1e-11 * max(abs(ref["Y0"]), 1e-300)
    # outputs left out of the loss get zero cotangents
    leaves2 = [t.clone().requires_grad_(True) for t in (st.pos, st.vel, st.rho, st.S)]
    outs2 = P.SphRhs.apply(*leaves2, mu.detach(), Y0.detach(), g, w.params, st.m)
    (outs2[0] * torch.as_tensor(cot["acc"]).cuda()).sum().backward()
    only = AD.rhs_vjp(w, {"acc": cot["acc"], "drho": np.zeros_like(cot["drho"]),
                          "dS": np.zeros_like(cot["dS"]), "rho_sum": np.zeros_like(cot["rho_sum"])})
    assert rel(leaves2[0].grad.cpu().numpy(), only["pos"]) < 1e-11


@pytest.mark.parametrize("case", ["single", "pair_at_h", "clumps"])
def test_rhs_adjoint_edge_sets(case):
    # one particle and a pair exactly h apart (no pair terms: only the density sum's
    # self term, which has no gradient); dense clumps with rows of up to 299 partners
    import test_gpu_forward as F
    h = 0.3
    pos = {"single": lambda: np.full((3, 1), 0.5),
           "pair_at_h": lambda: np.array([[0.0, h], [0.0, 0.0], [0.0, 0.0]]),
           "clumps": lambda: F.clumps(h)}[case]()
    w = F._state_on(pos, h, seed=53)
    rng = np.random.default_rng(5)
    ref_out = native.rhs_workload(w, want_L=False)
    cot = {k: rng.normal(size=ref_out[k].shape) for k in ref_out}
    st = gpu_state(w)
    for pairs in (False, True):
        g = P.sph_build_cells(st.pos, w.h, skin=0.01 * h, pairs=pairs)
        got = P.sph_rhs_adjoint(g, st, w.params, {k: torch.as_tensor(v).cuda() for k, v in cot.items()})
        assert P.workspace_status(got["_ws"]) == 0
        if case != "clumps":
            for k in ("pos", "vel", "rho", "S"):
                assert torch.all(got[k] == 0.0), k
            continue
        ref = AD.rhs_vjp(w, cot)
        for k in ("pos", "vel", "rho", "S"):
            assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k


@pytest.mark.parametrize("pairs", [False, True])
def test_rhs_adjoint_with_damage_matches_oracle(pairs):
    # a fixed damage field (section 2.7), densities on both sides of rho0: the adjoint
    # against the reverse-mode product of the oracle's transcription with the same field
    w = small("cube8_visc")
    rng = np.random.default_rng(17)
    w.d = rng.uniform(0.0, 1.0, w.n)
    w.d[rng.random(w.n) < 0.2] = 0.0
    w.d[rng.random(w.n) < 0.05] = 1.0
    w.rho = w.params["rho0"] * rng.uniform(0.995, 1.005, w.n)
    ref_out = native.rhs_workload(w, want_L=False)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ref_out}
    ref = AD.rhs_vjp(w, cot)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, d=w.d)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=pairs)
    got = P.sph_rhs_adjoint(g, st, w.params, {k: torch.as_tensor(v).cuda() for k, v in cot.items()})
    assert P.workspace_status(got["_ws"]) == 0
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    # the damage matters here
    w.d = None
    plain = AD.rhs_vjp(w, cot)
    assert rel(plain["rho"], ref["rho"]) > 1e-3


@pytest.mark.parametrize("variant", ["cells", "list", "corrected", "damage"])
def test_rhs_adjoint_murnaghan_matches_oracle(variant):
    # the Murnaghan equation (section 2.5.2): pressure slope and the per-particle sound
    # speed in Pi, against the reverse-mode product of the oracle's transcription
    w = small("cube8_visc")
    w.params.update(eos=1.0, n_M=4.0, correction=1.0 if variant == "corrected" else 0.0)
    rng = np.random.default_rng(19)
    w.rho = w.params["rho0"] * rng.uniform(0.97, 1.03, w.n)
    if variant == "damage":
        w.d = rng.uniform(0.0, 1.0, w.n)
    ref_out = native.rhs_workload(w, want_L=False)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ref_out}
    ref = AD.rhs_vjp(w, cot)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, d=getattr(w, "d", None))
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=variant != "cells")
    got = P.sph_rhs_adjoint(g, st, w.params, {k: torch.as_tensor(v).cuda() for k, v in cot.items()})
    assert P.workspace_status(got["_ws"]) == 0
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"])


@pytest.mark.parametrize("variant", ["cells", "list", "corrected", "damage_as", "extra"])
def test_rhs_adjoint_tillotson_matches_oracle(variant):
    # the Tillotson equation (section 2.5.3) over its three regions: gradients with
    # respect to rho and u through the pressure and through the sound speed (second
    # derivatives of p), against the oracle's reverse-mode product
    w = small("cube8_visc")
    w.params.update(eos=2.0, rho_cut=0.0, correction=1.0 if variant == "corrected" else 0.0)
    rng = np.random.default_rng(23)
    Eiv, Ecv = w.params["E_iv"], w.params["E_cv"]
    w.rho = w.params["rho0"] * rng.uniform(0.97, 1.03, w.n)
    w.u = rng.choice([0.5 * Eiv, 0.5 * (Eiv + Ecv), 1.3 * Ecv], w.n) * rng.uniform(0.95, 1.05, w.n)
    if variant == "damage_as":
        w.d = rng.uniform(0.0, 1.0, w.n)
        w.params.update(eps_s=0.2, n_s=4.0)
    if variant == "extra":
        w.params.update(xsph=0.5)
    ref_out = native.rhs_workload(w, want_L=False, want_extra=variant == "extra")
    keys = ("acc", "drho", "dS", "rho_sum") + (("du",) if variant == "extra" else ())
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in keys}
    if variant == "extra":
        cot["xv"] = rng.normal(size=(3, w.n)) / np.abs(ref_out["xv"] - w.vel).max()
    ref = AD.rhs_vjp(w, cot)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, u=w.u, d=getattr(w, "d", None))
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=variant != "cells")
    got = P.sph_rhs_adjoint(g, st, w.params, {k: torch.as_tensor(v).cuda() for k, v in cot.items()})
    assert P.workspace_status(got["_ws"]) == 0
    for k in ("pos", "vel", "rho", "S", "u"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    if variant == "cells":
        # the u gradient is not the pressure's alone: the sound speeds in Pi add to it
        assert np.abs(ref["u"]).max() > 0.0
        w0 = w.copy()
        w0.params.update(alpha=0.0, beta=0.0)
        ref0 = AD.rhs_vjp(w0, cot)
        assert rel(ref0["u"], ref["u"]) > 1e-6


def test_tillotson_adjoint_requires_the_u_gradient():
    w = small("cube10")
    w.params.update(eos=2.0)
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h)
    n = w.n
    out = {k: torch.empty(*sh, dtype=torch.float64).cuda() for k, sh in
           (("pos", (3, n)), ("vel", (3, n)), ("rho", (n,)), ("S", (6, n)))}
    fs = P.api.fields_struct(out["pos"], out["vel"], out["rho"], out["S"])
    acc = torch.ones(3, n, dtype=torch.float64).cuda()
    dc = L.DerivCot(acc[0].data_ptr(), acc[1].data_ptr(), acc[2].data_ptr())
    ws = P.workspace(L.SPH_OP_ADJOINT, n, 0)
    dp = torch.empty(2, dtype=torch.float64).cuda()
    cs = st.c_state()
    with pytest.raises(L.SphError) as e:
        L.check(L.lib().sph_rhs_adjoint(C.byref(g.c), C.byref(cs), C.byref(P.api.params_struct(w.params)),
                                        C.byref(dc), C.byref(fs), P.api._ptr(dp), P.api._ptr(ws),
                                        ws.numel(), P.api._stream()))
    assert e.value.code == L.SPH_ERR_INVALID_ARG


@pytest.mark.parametrize("variant", ["cells", "list", "corrected", "murnaghan_damage", "n2.5"])
def test_rhs_adjoint_artificial_stress_matches_oracle(variant):
    # the artificial stress (section 3.1.4) with half the particles in tension
    w = small("cube8_visc")
    w.params.update(eps_s=0.2, n_s=2.5 if variant == "n2.5" else 4.0,
                    correction=1.0 if variant == "corrected" else 0.0)
    rng = np.random.default_rng(23)
    w.rho = w.params["rho0"] * rng.uniform(0.99, 1.01, w.n)
    if variant == "murnaghan_damage":
        w.params.update(eos=1.0, n_M=4.0)
        w.d = rng.uniform(0.0, 1.0, w.n)
    ref_out = native.rhs_workload(w, want_L=False)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ref_out}
    ref = AD.rhs_vjp(w, cot)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, d=getattr(w, "d", None))
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=variant != "cells")
    got = P.sph_rhs_adjoint(g, st, w.params, {k: torch.as_tensor(v).cuda() for k, v in cot.items()})
    assert P.workspace_status(got["_ws"]) == 0
    for k in ("pos", "vel", "rho", "S"):
        assert rel(got[k].cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    w.params["eps_s"] = 0.0  # the artificial stress matters here
    assert rel(AD.rhs_vjp(w, cot)["pos"], ref["pos"]) > 1e-6


@pytest.mark.parametrize("variant", ["murnaghan", "artificial_stress", "both_corrected"])
def test_leapfrog_gradient_with_murnaghan_and_artificial_stress(variant):
    w = small("cube8_visc")
    rng = np.random.default_rng(29)
    w.rho = w.params["rho0"] * rng.uniform(0.99, 1.01, w.n)
    if variant in ("murnaghan", "both_corrected"):
        w.params.update(eos=1.0, n_M=4.0)
    if variant in ("artificial_stress", "both_corrected"):
        w.params.update(eps_s=0.2, n_s=4.0)
    if variant == "both_corrected":
        w.params.update(correction=1.0)
    steps = 8
    st, g, fin, ck = run_leapfrog(w, steps, pairs=True)
    cot = {"vel": (fin.vel * fin.m).contiguous()}
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, steps, ck, cot)
    assert P.workspace_status(got["_ws"]) == 0
    ref = AD.leapfrog_grad(w, steps, w.dt, "ke")
    assert rel(got["vel"].cpu().numpy(), ref["v0"]) < 1e-10
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-10 * abs(ref["mu"])


@pytest.mark.parametrize("variant", ["cells", "list", "corrected", "all_terms", "du_only", "xv_only"])
def test_rhs_adjoint_energy_and_xsph_cotangents(variant):
    # cotangents of du/dt (section 3.1.2) and of dx/dt with XSPH (section 3.1.5)
    w = small("cube8_visc")
    w.params.update(xsph=0.5, correction=1.0 if variant == "corrected" else 0.0)
    rng = np.random.default_rng(31)
    w.rho = w.params["rho0"] * rng.uniform(0.99, 1.01, w.n)
    if variant == "all_terms":
        w.params.update(eps_s=0.2, n_s=4.0, eos=1.0, n_M=4.0)
        w.d = rng.uniform(0.0, 1.0, w.n)
    ref_out = native.rhs_workload(w, want_L=False, want_extra=True)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max()
           for k in ("acc", "drho", "dS", "rho_sum")}
    cot["du"] = rng.normal(size=w.n) / np.abs(ref_out["du"]).max()
    cot["xv"] = rng.normal(size=(3, w.n)) / np.abs(ref_out["xv"] - w.vel).max()
    if variant == "du_only":
        cot = {"du": cot["du"]}
    if variant == "xv_only":
        cot = {"xv": cot["xv"]}
    ref = AD.rhs_vjp(w, cot)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, d=getattr(w, "d", None))
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=variant != "cells")
    got = P.sph_rhs_adjoint(g, st, w.params, {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()})
    assert P.workspace_status(got["_ws"]) == 0
    for k in ("pos", "vel", "rho", "S"):
        gk = got[k].cpu().numpy()
        if ref[k] is None:  # no dependence (the XSPH sum on the stress)
            assert np.all(gk == 0.0), k
            continue
        assert rel(gk, ref[k]) < 1e-11, k
    if ref["mu"] is not None and ref["mu"] != 0.0:
        assert abs(float(got["mu"]) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    # Y0 is reduced per wavefront on the list path, per block on the cell path
    y0 = 0.0 if ref["Y0"] is None else ref["Y0"]
    assert abs(float(got["Y0"]) - y0) <= 1e-11 * max(abs(y0), 1e-300), (float(got["Y0"]), y0)
    # bit-identical repeat (fixed reduction order, no atomics)
    again = P.sph_rhs_adjoint(g, st, w.params, {k: torch.as_tensor(v).cuda().contiguous() for k, v in cot.items()})
    for k in ("pos", "vel", "rho", "S", "mu", "Y0"):
        assert torch.equal(got[k], again[k]), k


def test_leapfrog_with_fixed_damage_trajectory_and_gradient():
    # a damage field held fixed over the trajectory (section 2.7): states and the
    # gradient of the final kinetic energy against the oracle's transcription
    w = small("cube8_visc")
    rng = np.random.default_rng(37)
    w.rho = w.params["rho0"] * rng.uniform(0.99, 1.01, w.n)
    w.d = rng.uniform(0.0, 1.0, w.n)
    steps = 8
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, d=w.d)
    g = P.sph_build_cells(st.pos, w.h, skin=0.5 * w.dx, pairs=True)
    fin, ck = P.sph_leapfrog(g, st, w.params, w.dt, steps)
    assert P.workspace_status(fin._ws) == 0
    pos, vel, rho, S, m, par = AD.as_tensors(w)
    with torch.no_grad():
        x, v, r, s = AD.leapfrog(pos, vel, rho, S, m, par, steps, w.dt, d=w.d)
    assert rel(fin.vel.cpu().numpy(), v.numpy()) < 1e-11
    assert rel(fin.S.cpu().numpy(), s.numpy()) < 1e-11
    cot = {"vel": (fin.vel * fin.m).contiguous()}
    got = P.sph_leapfrog_adjoint(g, st, w.params, w.dt, steps, ck, cot)
    assert P.workspace_status(got["_ws"]) == 0
    ref = AD.leapfrog_grad(w, steps, w.dt, "ke")
    assert rel(got["vel"].cpu().numpy(), ref["v0"]) < 1e-10
    assert abs(float(got["mu"]) - ref["mu"]) <= 1e-10 * abs(ref["mu"])
    # the damage matters on this trajectory
    w.d = None
    assert rel(AD.leapfrog_grad(w, steps, w.dt, "ke")["v0"], ref["v0"]) > 1e-6


def test_autograd_function_with_extra_outputs_and_damage():
    w = small("cube8_visc")
    w.params.update(xsph=0.5, eps_s=0.2, n_s=4.0)
    rng = np.random.default_rng(41)
    w.rho = w.params["rho0"] * rng.uniform(0.99, 1.01, w.n)
    w.d = rng.uniform(0.0, 1.0, w.n)
    ref_out = native.rhs_workload(w, want_L=False, want_extra=True)
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in ("acc", "drho", "dS", "rho_sum", "du")}
    cot["xv"] = rng.normal(size=(3, w.n)) / np.abs(ref_out["xv"] - w.vel).max()
    ref = AD.rhs_vjp(w, cot)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, d=w.d)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=True)
    leaves = [t.clone().requires_grad_(True) for t in (st.pos, st.vel, st.rho, st.S)]
    mu = torch.tensor(w.params["mu"], dtype=torch.float64, device="cuda", requires_grad=True)
    Y0 = torch.tensor(w.params["Y0"], dtype=torch.float64, device="cuda", requires_grad=True)
    outs = P.SphRhs.apply(*leaves, mu, Y0, g, w.params, st.m, st.d, True)
    assert len(outs) == 6
    loss = sum((o * torch.as_tensor(cot[k]).cuda()).sum()
               for k, o in zip(("acc", "drho", "dS", "rho_sum", "du", "xv"), outs))
    loss.backward()
    for k, t in zip(("pos", "vel", "rho", "S"), leaves):
        assert rel(t.grad.cpu().numpy(), ref[k]) < 1e-11, k
    assert abs(float(mu.grad) - ref["mu"]) <= 1e-11 * abs(ref["mu"])
    y0 = 0.0 if ref["Y0"] is None else ref["Y0"]
    assert abs(float(Y0.grad) - y0) <= 1e-11 * max(abs(y0), 1e-300), (float(Y0.grad), y0)


def test_autograd_function_refuses_inputs_changed_in_place():
    # the inputs are saved through autograd: an in-place change between forward and
    # backward raises instead of differentiating at the changed state
    w = small("cube8_visc")
    st = gpu_state(w)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=True)
    leaves = [t.clone().requires_grad_(True) for t in (st.pos, st.vel, st.rho, st.S)]
    x = leaves[0] * 1.0  # a non-leaf the caller can still modify in place
    mu = torch.tensor(w.params["mu"], dtype=torch.float64, device="cuda")
    Y0 = torch.tensor(w.params["Y0"], dtype=torch.float64, device="cuda")
    outs = P.SphRhs.apply(x, *leaves[1:], mu, Y0, g, w.params, st.m)
    with torch.no_grad():
        x.add_(1e-3 * w.dx)
    with pytest.raises(RuntimeError):
        outs[0].sum().backward()


def test_autograd_function_tillotson_gradient_of_u():
    w = small("cube8_visc")
    w.params.update(eos=2.0, rho_cut=0.0)
    rng = np.random.default_rng(43)
    Eiv, Ecv = w.params["E_iv"], w.params["E_cv"]
    w.rho = w.params["rho0"] * rng.uniform(0.97, 1.03, w.n)
    w.u = rng.choice([0.5 * Eiv, 0.5 * (Eiv + Ecv), 1.3 * Ecv], w.n) * rng.uniform(0.95, 1.05, w.n)
    ref_out = native.rhs_workload(w, want_L=False)
    keys = ("acc", "drho", "dS", "rho_sum")
    cot = {k: rng.normal(size=ref_out[k].shape) / np.abs(ref_out[k]).max() for k in keys}
    ref = AD.rhs_vjp(w, cot)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, u=w.u)
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, pairs=True)
    leaves = [t.clone().requires_grad_(True) for t in (st.pos, st.vel, st.rho, st.S)]
    u = st.u.clone().requires_grad_(True)
    mu = torch.tensor(w.params["mu"], dtype=torch.float64, device="cuda")
    Y0 = torch.tensor(w.params["Y0"], dtype=torch.float64, device="cuda")
    outs = P.SphRhs.apply(*leaves, mu, Y0, g, w.params, st.m, None, False, u)
    loss = sum((o * torch.as_tensor(cot[k]).cuda()).sum() for k, o in zip(keys, outs))
    loss.backward()
    for k, t in zip(("pos", "vel", "rho", "S"), leaves):
        assert rel(t.grad.cpu().numpy(), ref[k]) < 1e-11, k
    assert rel(u.grad.cpu().numpy(), ref["u"]) < 1e-11


def test_full_size_tillotson_u_gradient_matches_finite_differences():
    # two spheres, 262,144 particles, on the pair list as the step is timed: the
    # adjoint's directional derivative along u against central differences of the GPU
    # forward, u kept inside the Tillotson regions (the objective is smooth in u there)
    w = W.config(1)
    rng = np.random.default_rng(47)
    w.params.update(eos=2.0, rho_cut=0.0)
    Eiv, Ecv = w.params["E_iv"], w.params["E_cv"]
    w.rho = w.params["rho0"] * rng.uniform(0.98, 1.02, w.n)
    w.u = rng.choice([0.5 * Eiv, 0.5 * (Eiv + Ecv), 1.3 * Ecv], w.n) * rng.uniform(0.95, 1.05, w.n)
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, u=w.u)
    g = P.sph_build_cells(st.pos, w.h, skin=0.5 * w.dx, pairs=True)
    base = P.sph_rhs(g, st, w.params, "fp64")
    keys = ("acc", "drho", "dS")
    cot = {k: torch.randn_like(base[k]) / base[k].abs().max() for k in keys}
    got = P.sph_rhs_adjoint(g, st, w.params, cot)
    assert P.workspace_status(got["_ws"]) == 0
    dirn = torch.as_tensor(rng.normal(size=w.n)).cuda()
    ad = float((got["u"] * dirn).sum())
    e = 1e-6 * Ecv

    def objective(sign):
        s = P.ParticleState(st.pos, st.vel, st.rho, st.S, st.m, u=st.u + sign * e * dirn)
        o = P.sph_rhs(g, s, w.params, "fp64")
        return sum(float((o[k] * cot[k]).sum()) for k in keys)

    fd = (objective(+1) - objective(-1)) / (2 * e)
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    assert np.isfinite(got["rho"].cpu().numpy()).all()
