"""Torch-facing wrappers of the C ABI (same names as the C entry points).

All tensors live on the GPU in float64 (indices int32/int64), contiguous,
structure-of-arrays: positions and velocities (3, n), stress (6, n) in the
order xx, yy, zz, xy, xz, yz, density and mass (n,).  Calls are enqueued on
torch's current stream.  These functions only marshal arguments; the work is
done by libsph's kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

F64 = torch.float64
REC_DOUBLES = 16  # operand record of one slot (sph_deriv.rec, sph_deriv_cot.rec)
PARAM_ORDER = ("h", "rho0", "c", "mu", "Y0", "alpha", "beta", "eps_v", "rho_cut", "correction",
               "eps_s", "n_s", "dmpd", "xsph", "eos", "n_M", "a_T", "b_T", "A_T", "B_T", "E0_T",
               "alpha_T", "beta_T", "E_iv", "E_cv")
# parameters that may be left out of a dict: neutral values, and for the equations of
# state the liquid equation with aluminium 6061's Tillotson constants (section 4)
PARAM_DEFAULTS = {"correction": 0.0, "eps_s": 0.0, "n_s": 4.0, "dmpd": 0.0, "xsph": 0.0,
                  "eos": 0.0, "n_M": 4.0, "a_T": 0.5, "b_T": 1.63, "A_T": 75.2e9, "B_T": 65e9,
                  "E0_T": 5e6, "alpha_T": 5.0, "beta_T": 5.0, "E_iv": 3e6, "E_cv": 13.9e6}
DERIV_KEYS = ("acc", "drho", "dS", "rho_sum")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dev(t: torch.Tensor, dtype=F64) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("tensors must be on the GPU")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor")
    return t


@dataclass
class ParticleState:
    pos: torch.Tensor  # (3, n)
    vel: torch.Tensor  # (3, n)
    rho: torch.Tensor  # (n,)
    S: torch.Tensor    # (6, n)
    m: torch.Tensor    # (n,)
    u: torch.Tensor | None = None  # (n,) specific internal energy (Tillotson only)
    d: torch.Tensor | None = None  # (n,) damage
    flaw_ptr: torch.Tensor | None = None  # (n + 1,) int64 offsets of the flaw lists
    flaw_eps: torch.Tensor | None = None  # (flaw_ptr[n],) activation thresholds

    @property
    def n(self) -> int:
        return int(self.rho.shape[0])

    @classmethod
    def from_arrays(cls, pos, vel, rho, S, m, device="cuda", u=None, d=None, flaws=None):
        t = lambda a: torch.as_tensor(a, dtype=F64).to(device).contiguous() if a is not None else None
        fp = fe = None
        if flaws is not None:
            fp = torch.as_tensor(flaws[0], dtype=torch.int64).to(device).contiguous()
            fe = t(flaws[1])
        return cls(t(pos), t(vel), t(rho), t(S), t(m), t(u), t(d), fp, fe)

    def clone(self) -> "ParticleState":
        c = lambda t: t.clone() if t is not None else None
        return ParticleState(self.pos.clone(), self.vel.clone(), self.rho.clone(), self.S.clone(),
                             self.m.clone(), c(self.u), c(self.d), c(self.flaw_ptr), c(self.flaw_eps))

    def c_state(self) -> L.State:
        for t in (self.pos, self.vel, self.rho, self.S, self.m):
            _dev(t)
        n = self.n
        assert self.pos.shape == (3, n) and self.vel.shape == (3, n) and self.S.shape == (6, n)
        for t in (self.u, self.d):
            if t is not None:
                _dev(t)
                assert t.shape == (n,)
        if self.flaw_ptr is not None:
            _dev(self.flaw_ptr, torch.int64)
            _dev(self.flaw_eps)
            assert self.flaw_ptr.shape == (n + 1,)
        p, v, s = self.pos, self.vel, self.S
        q = lambda t: t.data_ptr() if t is not None else None
        return L.State(n, p[0].data_ptr(), p[1].data_ptr(), p[2].data_ptr(), v[0].data_ptr(),
                       v[1].data_ptr(), v[2].data_ptr(), self.rho.data_ptr(), s[0].data_ptr(),
                       s[1].data_ptr(), s[2].data_ptr(), s[3].data_ptr(), s[4].data_ptr(),
                       s[5].data_ptr(), self.m.data_ptr(), q(self.u), q(self.d), q(self.flaw_ptr),
                       q(self.flaw_eps))


def params_struct(params) -> L.Params:
    if isinstance(params, dict):
        vals = [float(params.get(k, PARAM_DEFAULTS[k])) if k in PARAM_DEFAULTS else float(params[k])
                for k in PARAM_ORDER]
    else:
        vals = [float(v) for v in params]
    return L.Params(*vals)


def workspace(op: int, n: int, ncells: int = 0, device="cuda") -> torch.Tensor:
    """Caller-owned scratch buffer for one operation."""
    return torch.empty(L.workspace_bytes(op, n, ncells), dtype=torch.uint8, device=device)


def workspace_status(ws: torch.Tensor) -> int:
    """Synchronises and returns the workspace's device flag (0 = fine)."""
    rc = L.lib().sph_workspace_status(_ptr(ws), _stream())
    return int(rc)


class CellGrid:
    """Device cell list (keeps the tensors behind the C struct alive), optionally with a
    frozen candidate-pair list attached by sph_build_pairs."""

    def __init__(self, perm, cell_start, cell_of, cstruct: L.Grid):
        self.perm, self.cell_start, self.cell_of, self.c = perm, cell_start, cell_of, cstruct
        self.ws = None
        self.pairs = None  # (L.Pairs, count, block_start, slot, x0, partners) when attached

    @property
    def has_pairs(self) -> bool:
        return self.pairs is not None

    @property
    def n(self):
        return int(self.c.n)

    @property
    def dims(self):
        return tuple(self.c.dims)

    @property
    def h(self):
        return float(self.c.h)


def default_box(pos: torch.Tensor, h: float, skin: float = 0.0):
    lo = pos.min(dim=1).values.double().cpu().numpy() - (h + skin)
    hi = pos.max(dim=1).values.double().cpu().numpy() + (h + skin)
    return lo, hi


def sph_build_cells(pos: torch.Tensor, h: float, skin: float = 0.0, cells_per_h: int = 1,
                    box=None, ws: torch.Tensor | None = None, pairs: bool = False) -> CellGrid:
    """Bin particles into the cell grid (C: sph_build_cells); with ``pairs`` also attach
    the frozen candidate-pair list (C: sph_build_pairs)."""
    _dev(pos)
    n = int(pos.shape[1])
    lo, hi = default_box(pos, h, skin) if box is None else box
    dims, ncells, cell = L.grid_geometry(lo, hi, h, skin, cells_per_h)
    dev = pos.device
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    cell_of = torch.empty(n, dtype=torch.int32, device=dev)
    cell_start = torch.empty(ncells + 1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(L.SPH_OP_BUILD, n, ncells, dev)
    g = L.Grid()
    lo_a = (C.c_double * 3)(*[float(v) for v in lo])
    hi_a = (C.c_double * 3)(*[float(v) for v in hi])
    L.check(L.lib().sph_build_cells(_ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]), n, lo_a, hi_a,
                                    float(h), float(skin), int(cells_per_h), _ptr(perm),
                                    _ptr(cell_start), ncells, _ptr(cell_of), C.byref(g), _ptr(ws),
                                    ws.numel(), _stream()))
    grid = CellGrid(perm, cell_start, cell_of, g)
    grid.ws = ws
    if pairs:
        sph_build_pairs(grid, pos)
    return grid


def sph_build_pairs(grid: CellGrid, pos: torch.Tensor, capacity: int | None = None,
                    ws: torch.Tensor | None = None) -> int:
    """Attach a frozen candidate-pair list (radius h + skin of the grid) built at ``pos``
    (C: sph_build_pairs).  Returns the number of list entries.  Synchronises once."""
    _dev(pos)
    n = grid.n
    dev = pos.device
    nb = (n + 63) // 64
    count = torch.empty(n, dtype=torch.int32, device=dev)
    partners = torch.empty(n, dtype=torch.int32, device=dev)
    block_start = torch.empty(nb + 1, dtype=torch.int64, device=dev)
    x0 = torch.empty(3 * n, dtype=F64, device=dev)
    if ws is None:
        ws = workspace(L.SPH_OP_PAIRS, n, 0, dev)
    needed = C.c_int64()
    out = L.Pairs()
    if capacity is None:
        rc = L.lib().sph_build_pairs(C.byref(grid.c), _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]),
                                     C.byref(out), _ptr(count), _ptr(partners), _ptr(block_start),
                                     C.c_void_p(0), 0,
                                     _ptr(x0), C.byref(needed), _ptr(ws), ws.numel(), _stream())
        if rc not in (L.SPH_OK, L.SPH_ERR_CAPACITY):
            L.check(rc)
        capacity = int(needed.value)
    slot = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    L.check(L.lib().sph_build_pairs(C.byref(grid.c), _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]),
                                    C.byref(out), _ptr(count), _ptr(partners), _ptr(block_start),
                                    _ptr(slot), capacity, _ptr(x0), C.byref(needed), _ptr(ws),
                                    ws.numel(), _stream()))
    grid.pairs = (out, count, block_start, slot, x0, partners)
    grid.c.pairs = C.cast(C.pointer(out), C.c_void_p)
    return int(needed.value)


def sph_neighbours(grid: CellGrid, pos: torch.Tensor, h: float, col_cap: int | None = None,
                   ws: torch.Tensor | None = None):
    """Partner lists as CSR (row_ptr int64 [n+1], col int32 [nnz]), rows ascending
    (C: sph_neighbours).  Synchronises once."""
    _dev(pos)
    n = grid.n
    dev = pos.device
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    if ws is None:
        ws = workspace(L.SPH_OP_NEIGHBOURS, n, 0, dev)
    nnz = C.c_int64()
    if col_cap is None:
        # first pass learns nnz (capacity 0), second fills
        rc = L.lib().sph_neighbours(C.byref(grid.c), _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]),
                                    float(h), _ptr(row_ptr), C.c_void_p(0), 0, C.byref(nnz),
                                    _ptr(ws), ws.numel(), _stream())
        if rc not in (L.SPH_OK, L.SPH_ERR_CAPACITY):
            L.check(rc)
        col_cap = int(nnz.value)
    col = torch.empty(max(col_cap, 1), dtype=torch.int32, device=dev)
    L.check(L.lib().sph_neighbours(C.byref(grid.c), _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]),
                                   float(h), _ptr(row_ptr), _ptr(col), col_cap, C.byref(nnz),
                                   _ptr(ws), ws.numel(), _stream()))
    return row_ptr, col[: int(nnz.value)]


def sph_gravity(pos: torch.Tensor, m: torch.Tensor, G: float, theta: float, eps: float = 0.0,
                count: bool = False, node_cap: int = 0, ws: torch.Tensor | None = None) -> dict:
    """Barnes-Hut monopole self-gravity (C: sph_gravity): dict acc (3, n), nodes (inner
    nodes of the tree) and, with ``count``, count (n, int32) bodies per particle.
    Synchronises once; retries once with the reported capacity when the tree outgrows
    ``node_cap`` (0: 2 n)."""
    _dev(pos)
    _dev(m)
    n = int(m.shape[0])
    assert pos.shape == (3, n)
    dev = m.device
    acc = torch.empty(3, n, dtype=F64, device=dev)
    cnt = torch.empty(n, dtype=torch.int32, device=dev) if count else None
    nodes = C.c_int64()
    for attempt in range(2):
        if ws is None or attempt:
            ws = workspace(L.SPH_OP_GRAVITY, n, node_cap, dev)
        rc = L.lib().sph_gravity(_ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]), _ptr(m), n, float(G),
                                 float(theta), float(eps), _ptr(acc[0]), _ptr(acc[1]), _ptr(acc[2]),
                                 _ptr(cnt) if cnt is not None else None, node_cap, C.byref(nodes),
                                 _ptr(ws), ws.numel(), _stream())
        if rc == L.SPH_ERR_CAPACITY and attempt == 0:
            node_cap = int(nodes.value)
            continue
        L.check(rc)
        break
    out = dict(acc=acc, nodes=int(nodes.value), _ws=ws)
    if cnt is not None:
        out["count"] = cnt
    return out


def new_deriv(n: int, device="cuda", extra: bool = False, damage: bool = False,
              vgrad: int = 0, records: bool = False):
    """Output arrays of sph_rhs; with ``extra`` also du (n) and xv (3, n) = dx/dt, with
    ``damage`` dd3 (n) = d(d^(1/3))/dt and n_act (n, int32), with ``vgrad`` = 9 (15 with
    the correction tensor) the velocity-gradient handoff for sph_rhs_adjoint (vgrad,
    (n, vgrad): one row per slot, the grid's slot order), with ``records`` the operand
    records for sph_rhs_adjoint (rec, (n, 16))."""
    d = dict(acc=torch.empty(3, n, dtype=F64, device=device),
             drho=torch.empty(n, dtype=F64, device=device),
             dS=torch.empty(6, n, dtype=F64, device=device),
             rho_sum=torch.empty(n, dtype=F64, device=device))
    if extra:
        d["du"] = torch.empty(n, dtype=F64, device=device)
        d["xv"] = torch.empty(3, n, dtype=F64, device=device)
    if damage:
        d["dd3"] = torch.empty(n, dtype=F64, device=device)
        d["n_act"] = torch.empty(n, dtype=torch.int32, device=device)
    if vgrad:
        d["vgrad"] = torch.empty(n, vgrad, dtype=F64, device=device)
    if records:
        d["rec"] = torch.empty(n, REC_DOUBLES, dtype=F64, device=device)
    return d


def deriv_struct(d: dict, cls=L.Deriv):
    a, s = d["acc"], d["dS"]
    for t in (a, s, d["drho"]):
        _dev(t)
    rs = d.get("rho_sum")
    p = lambda t: t.data_ptr() if t is not None else None
    args = [a[0].data_ptr(), a[1].data_ptr(), a[2].data_ptr(), d["drho"].data_ptr(),
            s[0].data_ptr(), s[1].data_ptr(), s[2].data_ptr(), s[3].data_ptr(),
            s[4].data_ptr(), s[5].data_ptr(), p(rs)]
    if cls is L.Deriv:
        du, xv = d.get("du"), d.get("xv")
        for t in (du, xv):
            if t is not None:
                _dev(t)
        args += [p(du)] + ([xv[0].data_ptr(), xv[1].data_ptr(), xv[2].data_ptr()]
                           if xv is not None else [None, None, None])
        dd3, na = d.get("dd3"), d.get("n_act")
        if dd3 is not None:
            _dev(dd3)
        if na is not None:
            _dev(na, torch.int32)
        vg, rec = d.get("vgrad"), d.get("rec")
        for t in (vg, rec):
            if t is not None:
                _dev(t)
        if rec is not None and (tuple(rec.shape) != (a.shape[1], REC_DOUBLES) or not rec.is_contiguous()):
            raise ValueError(f"rec must be contiguous ({a.shape[1]}, {REC_DOUBLES})")
        args += [p(dd3), p(na), p(vg), p(rec)]
    return cls(*args)


def fields_struct(pos, vel, rho, S, cls=L.Fields):
    return cls(pos[0].data_ptr(), pos[1].data_ptr(), pos[2].data_ptr(), vel[0].data_ptr(),
               vel[1].data_ptr(), vel[2].data_ptr(), rho.data_ptr(), S[0].data_ptr(),
               S[1].data_ptr(), S[2].data_ptr(), S[3].data_ptr(), S[4].data_ptr(),
               S[5].data_ptr())


def precision_code(precision) -> int:
    if precision in (L.SPH_FP64, "fp64", "f64"):
        return L.SPH_FP64
    if precision in (L.SPH_FP32_COMP, "fp32comp", "fp32_comp", "f32c"):
        return L.SPH_FP32_COMP
    raise ValueError(precision)


def sph_rhs(grid: CellGrid, state: ParticleState, params, precision="fp64", out=None,
            ws: torch.Tensor | None = None, extra: bool = False, damage: bool = False,
            vgrad: bool = False, records: bool = False) -> dict:
    """Right-hand side (C: sph_rhs): dict acc (3, n), drho (n), dS (6, n), rho_sum (n);
    with ``extra`` (or an ``out`` holding them) also du (n) and xv (3, n) = dx/dt, with
    ``damage`` the damage model's dd3 (n) and n_act (n) (the state's flaw lists needed),
    with ``vgrad`` (FP64) the velocity gradient and with ``records`` the operand records
    (rec) that sph_rhs_adjoint can take back."""
    n = state.n
    if out is None:
        nv = (15 if params_struct(params).correction != 0.0 else 9) if vgrad else 0
        out = new_deriv(n, state.rho.device, extra, damage, nv, records)
    if ws is None:
        ws = workspace(L.SPH_OP_RHS, n, 0, state.rho.device)
    cs = state.c_state()
    d = deriv_struct(out)
    L.check(L.lib().sph_rhs(C.byref(grid.c), C.byref(cs), C.byref(params_struct(params)),
                            precision_code(precision), C.byref(d), _ptr(ws), ws.numel(),
                            _stream()))
    out["_ws"] = ws
    return out


def sph_rhs_noalloc(grid: CellGrid, state: ParticleState, params, precision="fp64",
                    out=None, status: torch.Tensor | None = None) -> dict:
    """sph_rhs on the library's static scratch instead of a workspace (C: sph_rhs_noalloc);
    at most SPH_NOALLOC_MAX_N particles.  ``status`` (int32 device tensor of one element,
    optional) receives the device flag.  Calls that overlap on one GPU race."""
    n = state.n
    if out is None:
        out = new_deriv(n, state.rho.device)
    if status is not None:
        _dev(status, torch.int32)
    cs = state.c_state()
    d = deriv_struct(out)
    L.check(L.lib().sph_rhs_noalloc(C.byref(grid.c), C.byref(cs), C.byref(params_struct(params)),
                                    precision_code(precision), C.byref(d), _ptr(status), _stream()))
    return out


def sph_rhs_adjoint(grid: CellGrid, state: ParticleState, params, cot: dict,
                    ws: torch.Tensor | None = None, vgrad: torch.Tensor | None = None,
                    rec: torch.Tensor | None = None) -> dict:
    """Vector-Jacobian product of sph_rhs (C: sph_rhs_adjoint).  ``cot`` has keys of
    sph_rhs's outputs (acc, drho, dS, rho_sum, du, xv; missing = zero).  ``vgrad``: the
    "vgrad" output of an FP64 sph_rhs on the same grid, state and params, reused instead
    of forming the velocity gradient again; ``rec`` likewise its "rec" output (the
    operand records), reused instead of running the prepass again.  Returns gradients
    pos, vel, rho, S, mu, Y0, and u with the Tillotson equation."""
    n = state.n
    dev = state.rho.device
    z3 = lambda k, shape: _dev(cot[k]) if cot.get(k) is not None else None
    acc, drho, dS, rs = (z3("acc", None), z3("drho", None), z3("dS", None), z3("rho_sum", None))
    du, xv = z3("du", None), z3("xv", None)
    p = lambda t, i=None: (t[i].data_ptr() if i is not None else t.data_ptr()) if t is not None else None
    if vgrad is not None:
        _dev(vgrad)
        want = 15 if params_struct(params).correction != 0.0 else 9
        if tuple(vgrad.shape) != (n, want) or not vgrad.is_contiguous():
            raise ValueError(f"vgrad must be contiguous ({n}, {want}), got {tuple(vgrad.shape)}")
    if rec is not None:
        _dev(rec)
        if tuple(rec.shape) != (n, REC_DOUBLES) or not rec.is_contiguous():
            raise ValueError(f"rec must be contiguous ({n}, {REC_DOUBLES}), got {tuple(rec.shape)}")
    dc = L.DerivCot(p(acc, 0), p(acc, 1), p(acc, 2), p(drho), p(dS, 0), p(dS, 1), p(dS, 2),
                    p(dS, 3), p(dS, 4), p(dS, 5), p(rs), p(du), p(xv, 0), p(xv, 1), p(xv, 2),
                    p(vgrad), p(rec))
    g = dict(pos=torch.empty(3, n, dtype=F64, device=dev), vel=torch.empty(3, n, dtype=F64, device=dev),
             rho=torch.empty(n, dtype=F64, device=dev), S=torch.empty(6, n, dtype=F64, device=dev))
    dparams = torch.empty(2, dtype=F64, device=dev)
    if ws is None:
        ws = workspace(L.SPH_OP_ADJOINT, n, 0, dev)
    cs = state.c_state()
    fs = fields_struct(g["pos"], g["vel"], g["rho"], g["S"])
    if params_struct(params).eos == 2.0:
        g["u"] = torch.empty(n, dtype=F64, device=dev)
        fs.u = g["u"].data_ptr()
    L.check(L.lib().sph_rhs_adjoint(C.byref(grid.c), C.byref(cs), C.byref(params_struct(params)),
                                    C.byref(dc), C.byref(fs), _ptr(dparams), _ptr(ws), ws.numel(),
                                    _stream()))
    g["mu"] = dparams[0]
    g["Y0"] = dparams[1]
    g["_ws"] = ws
    return g


class SphRhs(torch.autograd.Function):
    """Differentiable FP64 right-hand side: forward calls sph_rhs, backward calls
    sph_rhs_adjoint (the exact vector-Jacobian product on the same partner set).

    apply(pos, vel, rho, S, mu, Y0, grid, params, m, d=None, extra=False, u=None)
    -> (acc, drho, dS, rho_sum), and with ``extra`` also (du, xv), the energy rate and
    dx/dt with XSPH.  ``u`` (n), the specific internal energy read by the Tillotson
    equation, is differentiable too (its gradient comes from the adjoint).  pos, vel (3, n), rho (n), S (6, n), m (n) are device tensors in
    user order and mu, Y0 scalar tensors (their values replace params' mu and Y0; their
    gradients come from the adjoint).  The masses, a damage field d (n) and the other
    constants are held fixed."""

    @staticmethod
    def forward(ctx, pos, vel, rho, S, mu, Y0, grid, params, m, d=None, extra=False, u=None):
        p = dict(params) if isinstance(params, dict) else dict(zip(PARAM_ORDER, params))
        p["mu"] = float(mu)
        p["Y0"] = float(Y0)
        st = ParticleState(pos.detach().contiguous(), vel.detach().contiguous(),
                           rho.detach().contiguous(), S.detach().contiguous(), m.contiguous(),
                           u=None if u is None else u.detach().contiguous(),
                           d=None if d is None else d.detach().contiguous())
        out = sph_rhs(grid, st, p, "fp64", extra=extra, vgrad=True, records=True)
        # the inputs are saved through autograd, so that an in-place change between
        # forward and backward raises instead of differentiating at a changed state;
        # the velocity gradient and the operand records are kept for the backward,
        # which then forms neither again
        ctx.save_for_backward(pos, vel, rho, S, m, u, d)
        ctx.vgrad = out["vgrad"]
        ctx.rec = out["rec"]
        ctx.grid, ctx.params, ctx.extra = grid, p, extra
        ctx.mu_like, ctx.Y0_like = torch.as_tensor(mu), torch.as_tensor(Y0)
        res = (out["acc"], out["drho"], out["dS"], out["rho_sum"])
        return res + ((out["du"], out["xv"]) if extra else ())

    @staticmethod
    def backward(ctx, *grads):
        pos, vel, rho, S, m, u, d = ctx.saved_tensors
        c = lambda t: None if t is None else t.detach().contiguous()
        st = ParticleState(c(pos), c(vel), c(rho), c(S), c(m), u=c(u), d=c(d))
        names = ("acc", "drho", "dS", "rho_sum", "du", "xv")
        cot = {k: (v.contiguous() if v is not None else None) for k, v in zip(names, grads)}
        g = sph_rhs_adjoint(ctx.grid, st, ctx.params, cot, vgrad=ctx.vgrad, rec=ctx.rec)
        gmu = g["mu"].to(ctx.mu_like.device, ctx.mu_like.dtype).reshape(ctx.mu_like.shape)
        gY0 = g["Y0"].to(ctx.Y0_like.device, ctx.Y0_like.dtype).reshape(ctx.Y0_like.shape)
        return (g["pos"], g["vel"], g["rho"], g["S"], gmu, gY0, None, None, None, None, None,
                g.get("u"))


def _fields(n, dev):
    return dict(pos=torch.empty(3, n, dtype=F64, device=dev), vel=torch.empty(3, n, dtype=F64, device=dev),
                rho=torch.empty(n, dtype=F64, device=dev), S=torch.empty(6, n, dtype=F64, device=dev))


def sph_leapfrog(grid: CellGrid, state: ParticleState, params, dt: float, steps: int,
                 checkpoints: bool | torch.Tensor = True, out: ParticleState | None = None,
                 ws: torch.Tensor | None = None):
    """Kick-drift-kick trajectory of ``steps`` steps on the (frozen) grid (C: sph_leapfrog).
    Returns (final ParticleState, checkpoint tensor or None)."""
    n = state.n
    dev = state.rho.device
    if out is None:
        out = ParticleState(torch.empty_like(state.pos), torch.empty_like(state.vel),
                            torch.empty_like(state.rho), torch.empty_like(state.S), state.m)
    if checkpoints is True:
        ck = torch.empty(L.checkpoint_bytes(n, steps) // 8, dtype=F64, device=dev)
    elif checkpoints is False or checkpoints is None:
        ck = None
    else:
        ck = checkpoints
    if ws is None:
        ws = workspace(L.SPH_OP_LEAPFROG, n, 0, dev)
    cs = state.c_state()
    fs = fields_struct(out.pos, out.vel, out.rho, out.S)
    L.check(L.lib().sph_leapfrog(C.byref(grid.c), C.byref(cs), C.byref(params_struct(params)),
                                 float(dt), int(steps), C.byref(fs), _ptr(ck), _ptr(ws), ws.numel(),
                                 _stream()))
    out._ws = ws
    return out, ck


def sph_leapfrog_adjoint(grid: CellGrid, state0: ParticleState, params, dt: float, steps: int,
                         checkpoints: torch.Tensor, cot_final: dict, ws: torch.Tensor | None = None,
                         grad: dict | None = None) -> dict:
    """Gradient of <cot_final, final state> with respect to the initial state and (mu, Y0)
    (C: sph_leapfrog_adjoint).  ``cot_final`` keys pos, vel, rho, S (missing = zero)."""
    n = state0.n
    dev = state0.rho.device
    g = _fields(n, dev) if grad is None else grad
    dparams = torch.empty(2, dtype=F64, device=dev)
    if ws is None:
        ws = workspace(L.SPH_OP_LEAPFROG_ADJOINT, n, 0, dev)
    t = lambda k: _dev(cot_final[k]) if cot_final.get(k) is not None else None
    cp, cv, cr, cS = t("pos"), t("vel"), t("rho"), t("S")
    p = lambda x, i=None: (x[i].data_ptr() if i is not None else x.data_ptr()) if x is not None else None
    cf = L.CFields(p(cp, 0), p(cp, 1), p(cp, 2), p(cv, 0), p(cv, 1), p(cv, 2), p(cr),
                   p(cS, 0), p(cS, 1), p(cS, 2), p(cS, 3), p(cS, 4), p(cS, 5))
    cs = state0.c_state()
    fs = fields_struct(g["pos"], g["vel"], g["rho"], g["S"])
    L.check(L.lib().sph_leapfrog_adjoint(C.byref(grid.c), C.byref(cs), C.byref(params_struct(params)),
                                         float(dt), int(steps), _ptr(checkpoints), C.byref(cf),
                                         C.byref(fs), _ptr(dparams), _ptr(ws), ws.numel(), _stream()))
    g["mu"] = dparams[0]
    g["Y0"] = dparams[1]
    g["_ws"] = ws
    return g
