"""Pins of the corrected velocity gradient (section 3.1.6, linear consistency).

With C the inverse of M = sum_b V_b (x_b - x_a) (x) grad_a W_ab, the corrected
gradient sum_b V_b (v_b - v_a) (x) grad_a W_ab C reproduces every linear velocity
field v = A x + b exactly (A M C = A), at every particle whose M is regular,
including those at the free surface where the standard gradient is off; the
lattice factor of the standard gradient becomes exactly one.  None of these
re-types the oracle's formulas.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import autodiff as AD
from oracle import native

MU, Y0 = 2.7e10, 3e8


def body(n_side=7, jitter=0.1, seed=3, **over):
    return W.cube(n_side, 0.1, seed=seed, jitter=jitter, state="rest", correction=1.0, **over)


def L_of(w):
    return native.rhs_workload(w)["L"].reshape(3, 3, -1)


@pytest.mark.parametrize("jitter", [0.0, 0.1])
def test_linear_field_exact_everywhere(jitter):
    w = body(jitter=jitter)
    rng = np.random.default_rng(5)
    A = rng.normal(size=(3, 3)) * 100.0
    w.vel = np.ascontiguousarray(A @ w.pos + rng.normal(size=(3, 1)))
    L = L_of(w)
    assert np.abs(L - A[:, :, None]).max() < 1e-9 * np.abs(A).max()
    # the standard gradient misses it at the surface (the pin has teeth)
    w.params["correction"] = 0.0
    L0 = L_of(w)
    assert np.abs(L0 - A[:, :, None]).max() > 0.1 * np.abs(A).max()


def test_rigid_rotation_without_lattice_factor():
    # v = omega z x (x - c): corrected L is exactly the spin tensor at every particle,
    # so the strain rate vanishes and dS = R S~ - S~ R with R = L
    w = body(jitter=0.05)
    om, s = 20.0, 5e7
    c = w.pos.mean(1, keepdims=True)
    w.vel[0] = -om * (w.pos[1] - c[1])
    w.vel[1] = om * (w.pos[0] - c[0])
    w.S[0], w.S[1] = s, -s
    out = native.rhs_workload(w)
    L = out["L"].reshape(3, 3, -1)
    Om = np.zeros((3, 3))
    Om[1, 0], Om[0, 1] = om, -om
    assert np.abs(L - Om[:, :, None]).max() < 1e-9 * om
    dS = out["dS"]
    assert np.allclose(dS[3], 2 * om * s, rtol=1e-8)  # f_Y = 1 for s < Y0 / sqrt(3)
    assert np.abs(dS[[0, 1, 2, 4, 5]]).max() < 1e-8 * abs(s * om)


def test_singular_moment_matrix_keeps_standard_gradient():
    # two particles: M has rank one, so the correction is not applied
    w = W.two_particles((0.0, 0.0, 0.0), (0.3, 0.1, 0.0), va=(1.0, 2.0, 0.0), vb=(-3.0, 0.5, 1.0),
                        correction=1.0)
    L1 = L_of(w)
    w.params["correction"] = 0.0
    L0 = L_of(w)
    assert np.array_equal(L1, L0)


def test_continuity_and_momentum_unchanged():
    # the correction acts on the strain and rotation rates only
    w = body(jitter=0.1)
    rng = np.random.default_rng(9)
    w.vel = rng.normal(size=w.vel.shape) * 50.0
    w.rho = 2700.0 * (1 + 0.01 * rng.normal(size=w.n))
    a = native.rhs_workload(w)
    w.params["correction"] = 0.0
    b = native.rhs_workload(w)
    for k in ("acc", "drho", "rho_sum"):
        assert np.array_equal(a[k], b[k]), k
    assert not np.allclose(a["dS"], b["dS"])


def test_torch_transcription_matches_c_oracle_with_correction():
    w = body(jitter=0.1, alpha=1.0, beta=1.0)
    rng = np.random.default_rng(2)
    w.vel = rng.normal(size=w.vel.shape) * 50.0
    w.S = rng.normal(size=w.S.shape) * 1e7
    ref = native.rhs_workload(w)
    out = AD.rhs(*AD.as_tensors(w))
    for k in ("acc", "drho", "dS", "rho_sum"):
        a, b = ref[k], out[k].numpy()
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), k
    assert np.abs(ref["L"] - out["L"].reshape(9, -1).numpy()).max() <= 1e-13 * np.abs(ref["L"]).max()


@pytest.mark.parametrize("which", ["pos", "vel", "rho"])
def test_corrected_vjp_matches_finite_differences(which):
    w = body(n_side=5, jitter=0.1, seed=7)
    rng = np.random.default_rng(4)
    w.vel = rng.normal(size=w.vel.shape) * 50.0
    w.S = rng.normal(size=w.S.shape) * 1e7
    w.rho = 2700.0 * (1 + 0.01 * rng.normal(size=w.n))
    ref = native.rhs_workload(w, want_L=False)
    y = {k: rng.normal(size=v.shape) / np.abs(v).max() for k, v in ref.items()}
    g = AD.rhs_vjp(w, y)
    base = {"pos": w.pos, "vel": w.vel, "rho": w.rho}[which]
    d = rng.normal(size=base.shape)
    e = {"pos": 1e-6 * w.dx, "vel": 1e-4, "rho": 1e-4}[which]

    def J(sign):
        w2 = w.copy()
        setattr(w2, which, base + sign * e * d)
        o = native.rhs_workload(w2, want_L=False)
        return sum(float((o[k] * y[k]).sum()) for k in y)

    fd = (J(+1) - J(-1)) / (2 * e)
    ad = float((g[which] * d).sum())
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
