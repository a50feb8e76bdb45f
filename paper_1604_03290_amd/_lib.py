"""ctypes binding of libsph (the C ABI declared in include/sph.h).

Argument marshalling only: tensors are passed as raw device pointers together
with torch's current HIP stream; every computation runs in the library's HIP
kernels.  The library must have been built (``__graft_entry__.build()`` or
``python paper_1604_03290_amd/build.py``); nothing falls back to another
implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK = 0
SPH_ERR_INVALID_ARG = -1
SPH_ERR_CAPACITY = -2
SPH_ERR_WORKSPACE = -3
SPH_ERR_HIP = -4
SPH_ERR_DOMAIN = -5
SPH_ERR_NOT_IMPLEMENTED = -6
SPH_ERR_STALE_GRID = -7

SPH_FP64 = 0
SPH_FP32_COMP = 1

SPH_OP_BUILD, SPH_OP_NEIGHBOURS, SPH_OP_RHS, SPH_OP_ADJOINT = 0, 1, 2, 3
SPH_OP_LEAPFROG, SPH_OP_LEAPFROG_ADJOINT, SPH_OP_PAIRS, SPH_OP_GRAVITY = 4, 5, 6, 7
SPH_NOALLOC_MAX_N = 262144  # include/sph.h

_NAMES = {0: "SPH_OK", -1: "SPH_ERR_INVALID_ARG", -2: "SPH_ERR_CAPACITY", -3: "SPH_ERR_WORKSPACE",
          -4: "SPH_ERR_HIP", -5: "SPH_ERR_DOMAIN", -6: "SPH_ERR_NOT_IMPLEMENTED",
          -7: "SPH_ERR_STALE_GRID"}

_vp = C.c_void_p
_pd = C.c_void_p  # device pointers travel as plain addresses


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Pairs(C.Structure):
    _fields_ = [("n", C.c_int64), ("radius", C.c_double), ("skin", C.c_double), ("count", _vp),
                ("block_start", _vp), ("slot", _vp), ("capacity", C.c_int64), ("x0", _vp),
                ("partners", _vp)]


class Grid(C.Structure):
    _fields_ = [("n", C.c_int64), ("dims", C.c_int32 * 3), ("ncells", C.c_int64),
                ("lo", C.c_double * 3), ("cell", C.c_double), ("h", C.c_double),
                ("skin", C.c_double), ("perm", _vp), ("cell_start", _vp), ("cell_of", _vp),
                ("pairs", _vp)]


class State(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, _pd) for k in
                                     ("x", "y", "z", "vx", "vy", "vz", "rho", "sxx", "syy", "szz",
                                      "sxy", "sxz", "syz", "m", "u", "d", "flaw_ptr",
                                      "flaw_eps")]


class Params(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("h", "rho0", "c", "mu", "Y0", "alpha", "beta", "eps_v", "rho_cut", "correction",
                 "eps_s", "n_s", "dmpd", "xsph", "eos", "n_M", "a_T", "b_T", "A_T", "B_T", "E0_T",
                 "alpha_T", "beta_T", "E_iv", "E_cv")]


_DERIV = ("ax", "ay", "az", "drho", "dsxx", "dsyy", "dszz", "dsxy", "dsxz", "dsyz", "rho_sum")
_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "sxx", "syy", "szz", "sxy", "sxz", "syz")


class Deriv(C.Structure):
    _fields_ = [(k, _pd) for k in _DERIV + ("du", "dx", "dy", "dz", "dd3", "n_act", "vgrad", "rec")]


class DerivCot(C.Structure):
    _fields_ = [(k, _pd) for k in _DERIV + ("du", "dx", "dy", "dz", "vgrad", "rec")]


class Fields(C.Structure):
    _fields_ = [(k, _pd) for k in _FIELDS + ("u",)]


class CFields(C.Structure):
    _fields_ = [(k, _pd) for k in _FIELDS]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950); there is no other implementation")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.sph_version.restype = C.c_char_p
        L.sph_last_error.restype = C.c_char_p
        L.sph_workspace_bytes.restype = C.c_size_t
        L.sph_workspace_bytes.argtypes = [C.c_int, C.c_int64, C.c_int64]
        L.sph_checkpoint_bytes.restype = C.c_size_t
        L.sph_checkpoint_bytes.argtypes = [C.c_int64, C.c_int]
        L.sph_grid_geometry.argtypes = [P(C.c_double), P(C.c_double), C.c_double, C.c_double,
                                        C.c_int, P(C.c_int32), P(C.c_int64), P(C.c_double)]
        L.sph_build_cells.argtypes = [_pd, _pd, _pd, C.c_int64, P(C.c_double), P(C.c_double),
                                      C.c_double, C.c_double, C.c_int, _pd, _pd, C.c_int64, _pd,
                                      P(Grid), _pd, C.c_size_t, _vp]
        L.sph_build_pairs.argtypes = [P(Grid), _pd, _pd, _pd, P(Pairs), _pd, _pd, _pd, _pd,
                                      C.c_int64, _pd, P(C.c_int64), _pd, C.c_size_t, _vp]
        L.sph_neighbours.argtypes = [P(Grid), _pd, _pd, _pd, C.c_double, _pd, _pd, C.c_int64,
                                     P(C.c_int64), _pd, C.c_size_t, _vp]
        L.sph_rhs.argtypes = [P(Grid), P(State), P(Params), C.c_int, P(Deriv), _pd, C.c_size_t,
                              _vp]
        L.sph_rhs_noalloc.argtypes = [P(Grid), P(State), P(Params), C.c_int, P(Deriv), _pd, _vp]
        L.sph_gravity.argtypes = [_pd, _pd, _pd, _pd, C.c_int64, C.c_double, C.c_double,
                                  C.c_double, _pd, _pd, _pd, _pd, C.c_int64, P(C.c_int64), _pd,
                                  C.c_size_t, _vp]
        L.sph_rhs_adjoint.argtypes = [P(Grid), P(State), P(Params), P(DerivCot), P(Fields), _pd,
                                      _pd, C.c_size_t, _vp]
        L.sph_leapfrog.argtypes = [P(Grid), P(State), P(Params), C.c_double, C.c_int, P(Fields),
                                   _pd, _pd, C.c_size_t, _vp]
        L.sph_leapfrog_adjoint.argtypes = [P(Grid), P(State), P(Params), C.c_double, C.c_int, _pd,
                                           P(CFields), P(Fields), _pd, _pd, C.c_size_t, _vp]
        L.sph_workspace_status.argtypes = [_pd, _vp]
        L.sph_timing_enable.argtypes = [C.c_int]
        L.sph_timing_read.argtypes = [C.c_char_p, P(C.c_double), P(C.c_int64)]
        _lib = L
    return _lib


def check(rc: int):
    if rc != SPH_OK:
        raise SphError(rc, lib().sph_last_error().decode())
    return rc


def version() -> str:
    return lib().sph_version().decode()


def workspace_bytes(op: int, n: int, ncells: int = 0) -> int:
    return int(lib().sph_workspace_bytes(op, n, ncells))


def checkpoint_bytes(n: int, steps: int) -> int:
    return int(lib().sph_checkpoint_bytes(n, steps))


def grid_geometry(lo, hi, h: float, skin: float = 0.0, cells_per_h: int = 1):
    lo_a = (C.c_double * 3)(*[float(v) for v in lo])
    hi_a = (C.c_double * 3)(*[float(v) for v in hi])
    dims = (C.c_int32 * 3)()
    ncells = C.c_int64()
    cell = C.c_double()
    check(lib().sph_grid_geometry(lo_a, hi_a, float(h), float(skin), int(cells_per_h), dims,
                                  C.byref(ncells), C.byref(cell)))
    return tuple(dims), int(ncells.value), float(cell.value)


def timing_enable(on: bool = True):
    check(lib().sph_timing_enable(1 if on else 0))


def timing_reset():
    check(lib().sph_timing_reset())


def timing_read(kernel: str):
    """(total milliseconds, launches) of a bracketed kernel since the last reset."""
    ms = C.c_double()
    cnt = C.c_int64()
    check(lib().sph_timing_read(kernel.encode(), C.byref(ms), C.byref(cnt)))
    return float(ms.value), int(cnt.value)
