"""sph_rhs_noalloc, the entry point for callers that cannot allocate, against sph_rhs
through the C ABI: bit-identical outputs (the same kernels) on two calls in a row, the
second on a smaller and ragged set, FP64 and FP32-compensated, pair-list and cell
paths; the device flag through its status output, cleared by the next call."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
import paper_1604_03290_amd as P
from paper_1604_03290_amd import _lib as L

pytestmark = pytest.mark.gpu

KEYS = ("acc", "drho", "dS", "rho_sum")


def noalloc(g, st, params, precision, out, status):
    cs = st.c_state()
    d = P.api.deriv_struct(out)
    return L.lib().sph_rhs_noalloc(C.byref(g.c), C.byref(cs), C.byref(P.api.params_struct(params)),
                                   P.api.precision_code(precision), C.byref(d), P.api._ptr(status),
                                   P.api._stream())


def compare(w, precision, pairs):
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, "cuda")
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, cells_per_h=2, pairs=pairs)
    ref = P.sph_rhs(g, st, w.params, precision)
    assert P.workspace_status(ref["_ws"]) == 0
    out = P.api.new_deriv(w.n)
    status = torch.full((1,), 123, dtype=torch.int32, device="cuda")
    L.check(noalloc(g, st, w.params, precision, out, status))
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    for k in KEYS:
        assert torch.equal(out[k], ref[k]), (w.name, precision, pairs, k)
    return g, st


@pytest.mark.parametrize("precision", ["fp64", "fp32comp"])
@pytest.mark.parametrize("pairs", [True, False])
def test_noalloc_matches_sph_rhs_on_two_calls(precision, pairs):
    big = W.config(1)  # 262,144 particles, the largest size the scratch serves
    assert big.n == L.SPH_NOALLOC_MAX_N
    compare(big, precision, pairs)
    small = W.cube(15, 1.0 / 16, seed=5)  # 3,375 particles: 52 full wavefronts and 47
    compare(small, precision, pairs)


def test_noalloc_status_reports_the_device_flag_and_is_cleared():
    w = W.config(0)
    w.rho[17] = -1.0  # non-positive density: DOMAIN
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, "cuda")
    g = P.sph_build_cells(st.pos, w.h, skin=0.05 * w.dx, cells_per_h=2, pairs=True)
    out = P.api.new_deriv(w.n)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.check(noalloc(g, st, w.params, "fp64", out, status))
    torch.cuda.synchronize()
    assert int(status.item()) == L.SPH_ERR_DOMAIN
    w2 = W.config(0)
    st2 = P.ParticleState.from_arrays(w2.pos, w2.vel, w2.rho, w2.S, w2.m, "cuda")
    g2 = P.sph_build_cells(st2.pos, w2.h, skin=0.05 * w2.dx, cells_per_h=2, pairs=True)
    L.check(noalloc(g2, st2, w2.params, "fp64", out, status))
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    # the binding, without a status
    got = P.sph_rhs_noalloc(g2, st2, w2.params, "fp64")
    ref = P.sph_rhs(g2, st2, w2.params, "fp64")
    for k in KEYS:
        assert torch.equal(got[k], ref[k]), k
