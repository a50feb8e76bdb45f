"""ctypes front end of the C oracle (``sph_oracle.c``, ``gravity.c``).  Test infrastructure.

Arrays are numpy float64 structure-of-arrays: pos/vel (3, n), S (6, n),
rho/m (n,).  ``par`` is the parameter vector {h, rho0, c, mu, Y0, alpha,
beta, eps_v, rho_cut}.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_d = C.c_double
_i64 = C.c_int64
_pd = C.POINTER(C.c_double)
_pi64 = C.POINTER(C.c_int64)
_pi32 = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_kernel.argtypes = [_d, _d, _pd, _pd]
        L.orc_count_neighbours.argtypes = [_i64, _pd, _d, _pi64, _i64, _pi64]
        L.orc_count_neighbours.restype = _i64
        L.orc_fill_neighbours.argtypes = [_i64, _pd, _d, _pi64, _i64, _pi64, _pi32]
        L.orc_ball.argtypes = [_i64, _pd, _pd, _d, _pi64, _i64]
        L.orc_ball.restype = _i64
        L.orc_prepass.argtypes = [_i64, _pd, _pd, _pd, _pd, _pd, _pd]
        L.orc_rhs.argtypes = [_i64, _pd, _pd, _pd, _pd, _pd, _pd, _pi64, _i64, _pi64, _pi32,
                              _pd, _pd, _pd, _pd, _pd]
        L.orc_rhs2.argtypes = [_i64, _pd, _pd, _pd, _pd, _pd, _pd, _pd, _pd, _pi64, _i64,
                               _pi64, _pi32, _pd, _pd, _pd, _pd, _pd, _pd, _pd]
        L.orc_prepass2.argtypes = [_i64, _pd, _pd, _pd, _pd, _pd, _pd, _pd, _pd, _pd]
        L.orc_eos.argtypes = [_i64, _pd, _pd, _pd, _pd, _pd]
        L.orc_gravity.argtypes = [_i64, _pd, _pd, _d, _d, _d, _pi64, _i64, _pd, _pi64, _pi32]
        L.orc_gravity.restype = _i64
        L.orc_gravity_tree.argtypes = [_i64, _pd, _pd, _i64, _pi32, _pi64, _pd, _pd]
        L.orc_gravity_tree.restype = _i64
        _lib = L
    return _lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_pd)


def _i64a(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_pi64)


def threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS or the core count)."""
    return int(lib().orc_threads())


def set_threads(k: int) -> None:
    """OpenMP threads for later calls (timing only)."""
    lib().orc_set_threads(int(k))


def kernel(r: float, h: float):
    """(W, dW/dr) of the cubic B-spline with support radius h."""
    W, dW = C.c_double(), C.c_double()
    lib().orc_kernel(float(r), float(h), C.byref(W), C.byref(dW))
    return W.value, dW.value


def neighbours(pos, h: float, targets=None):
    """Brute-force partner sets: (row_ptr int64 [nt+1], col int32 [nnz]), each row ascending."""
    pos, ppos = _f64(pos)
    n = pos.shape[1]
    if targets is None:
        nt, ptg, tg = n, None, None
    else:
        tg, ptg = _i64a(targets)
        nt = tg.shape[0]
    counts = np.zeros(nt, dtype=np.int64)
    lib().orc_count_neighbours(n, ppos, float(h), ptg, nt, counts.ctypes.data_as(_pi64))
    row_ptr = np.zeros(nt + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.zeros(int(row_ptr[-1]), dtype=np.int32)
    lib().orc_fill_neighbours(n, ppos, float(h), ptg, nt, row_ptr.ctypes.data_as(_pi64),
                              col.ctypes.data_as(_pi32))
    return row_ptr, col


def ball(pos, centre, radius: float) -> np.ndarray:
    """Ascending indices of particles strictly within ``radius`` of ``centre``."""
    pos, ppos = _f64(pos)
    n = pos.shape[1]
    c, pc = _f64(np.asarray(centre, dtype=np.float64).reshape(3))
    cnt = lib().orc_ball(n, ppos, pc, float(radius), None, 0)
    out = np.zeros(max(cnt, 1), dtype=np.int64)
    lib().orc_ball(n, ppos, pc, float(radius), out.ctypes.data_as(_pi64), cnt)
    return out[:cnt]


def prepass(rho, S, par):
    rho, prho = _f64(rho)
    S, pS = _f64(S)
    par, ppar = _f64(par)
    n = rho.shape[0]
    p = np.zeros(n)
    f = np.zeros(n)
    sig = np.zeros((6, n))
    lib().orc_prepass(n, prho, pS, ppar, p.ctypes.data_as(_pd), f.ctypes.data_as(_pd),
                      sig.ctypes.data_as(_pd))
    return dict(p=p, fy=f, sigma=sig)


def prepass2(rho, S, par, u=None, d=None):
    """Pressure, limiter factor, sound speed and the (damaged) stress sigma (6, n)."""
    rho, prho = _f64(rho)
    S, pS = _f64(S)
    par, ppar = _f64(par)
    pu = _f64(u)[1] if u is not None else None
    pd_ = _f64(d)[1] if d is not None else None
    n = rho.shape[0]
    p, f, cs = np.zeros(n), np.zeros(n), np.zeros(n)
    sig = np.zeros((6, n))
    lib().orc_prepass2(n, prho, pu, pd_, pS, ppar, p.ctypes.data_as(_pd), f.ctypes.data_as(_pd),
                       cs.ctypes.data_as(_pd), sig.ctypes.data_as(_pd))
    return dict(p=p, fy=f, cs=cs, sigma=sig)


def eos(rho, par, u=None):
    """(pressure, squared sound speed) of every particle (sections 2.5.1 to 2.5.3)."""
    rho, prho = _f64(rho)
    par, ppar = _f64(par)
    pu = _f64(u)[1] if u is not None else None
    p = np.zeros(rho.shape[0])
    c2 = np.zeros(rho.shape[0])
    lib().orc_eos(rho.shape[0], prho, pu, ppar, p.ctypes.data_as(_pd), c2.ctypes.data_as(_pd))
    return p, c2


def rhs(pos, vel, rho, S, m, par, targets=None, csr=None, want_L: bool = True,
        want_extra: bool = False, u=None, d=None):
    """Right-hand side for ``targets`` (all particles when None).

    ``csr`` = (row_ptr, col) partner lists of the targets; computed by brute
    force when omitted.  Returns dict acc (3, nt), drho (nt), dS (6, nt),
    rho_sum (nt) and L (9, nt); with ``want_extra`` also du (nt), the specific
    internal energy rate, and xv (3, nt), dx/dt with XSPH.  ``u``: specific internal
    energy (the Tillotson equation's second input; zero when None); ``d``: damage.
    """
    pos, ppos = _f64(pos)
    vel, pvel = _f64(vel)
    rho, prho = _f64(rho)
    S, pS = _f64(S)
    m, pm = _f64(m)
    par, ppar = _f64(par)
    n = rho.shape[0]
    if csr is None:
        csr = neighbours(pos, par[0], targets)
    row_ptr, col = csr
    row_ptr, prow = _i64a(row_ptr)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if targets is None:
        nt, ptg = n, None
    else:
        tg, ptg = _i64a(targets)
        nt = tg.shape[0]
    assert row_ptr.shape[0] == nt + 1
    acc = np.zeros((3, nt))
    drho = np.zeros(nt)
    dS = np.zeros((6, nt))
    rs = np.zeros(nt)
    L = np.zeros((9, nt)) if want_L else None
    du = np.zeros(nt) if want_extra else None
    xv = np.zeros((3, nt)) if want_extra else None
    pnull = lambda a: a.ctypes.data_as(_pd) if a is not None else None
    uarr = _f64(u) if u is not None else (None, None)
    darr = _f64(d) if d is not None else (None, None)
    lib().orc_rhs2(n, ppos, pvel, prho, uarr[1], darr[1], pS, pm, ppar, ptg, nt, prow,
                   col.ctypes.data_as(_pi32),
                   acc.ctypes.data_as(_pd), drho.ctypes.data_as(_pd), dS.ctypes.data_as(_pd),
                   rs.ctypes.data_as(_pd), pnull(L), pnull(du), pnull(xv))
    out = dict(acc=acc, drho=drho, dS=dS, rho_sum=rs)
    if want_L:
        out["L"] = L
    if want_extra:
        out["du"] = du
        out["xv"] = xv
    return out


def rhs_workload(w, targets=None, csr=None, want_L: bool = True, want_extra: bool = False):
    """``rhs`` on a ``workloads.Workload``."""
    return rhs(w.pos, w.vel, w.rho, w.S, w.m, w.param_vector(), targets, csr, want_L, want_extra,
               getattr(w, "u", None), getattr(w, "d", None))


def gravity(pos, m, G: float, theta: float, eps: float = 0.0, targets=None):
    """Barnes-Hut monopole gravity (section 3.3): dict acc (3, nt), count (nt),
    tie (nt, bool: the walk met a node where the printed test s / r < theta and its
    squared form s^2 < theta^2 r^2 round to different decisions) and nodes (the
    number of inner nodes) for ``targets`` (all particles when None); the tree always
    holds every particle."""
    pos, ppos = _f64(pos)
    m, pm = _f64(m)
    n = m.shape[0]
    if targets is None:
        nt, ptg = n, None
    else:
        tg, ptg = _i64a(targets)
        nt = tg.shape[0]
    acc = np.zeros((3, nt))
    cnt = np.zeros(nt, dtype=np.int64)
    tie = np.zeros(nt, dtype=np.int32)
    nn = lib().orc_gravity(n, ppos, pm, G, theta, eps, ptg, nt, acc.ctypes.data_as(_pd),
                           cnt.ctypes.data_as(_pi64), tie.ctypes.data_as(_pi32))
    return dict(acc=acc, count=cnt, tie=tie.astype(bool), nodes=int(nn))


def gravity_tree(pos, m):
    """The oracle's inner nodes: depth (k,), corner (k, 3) integer cube corner at
    that depth, mass (k,), com (k, 3)."""
    pos, ppos = _f64(pos)
    m, pm = _f64(m)
    n = m.shape[0]
    cap = 0
    while True:
        depth = np.zeros(max(cap, 1), dtype=np.int32)
        corner = np.zeros((max(cap, 1), 3), dtype=np.int64)
        mass = np.zeros(max(cap, 1))
        com = np.zeros((max(cap, 1), 3))
        nn = lib().orc_gravity_tree(n, ppos, pm, cap, depth.ctypes.data_as(_pi32),
                                    corner.ctypes.data_as(_pi64), mass.ctypes.data_as(_pd),
                                    com.ctypes.data_as(_pd))
        if nn <= cap:
            return dict(depth=depth[:nn], corner=corner[:nn], mass=mass[:nn], com=com[:nn])
        cap = int(nn)
