"""Gradient oracle.  Test infrastructure.

The right-hand side of the C oracle written once more with plain torch CPU
float64 operations over an explicit list of ordered pairs, so that reverse-mode
automatic differentiation supplies the exact vector-Jacobian product
J^T y of the method's definition (no hand derivation).  The same formulas and
readings as ``sph_oracle.c`` (see its header for the passages):

  kernel (section 3.1.1), liquid equation of state (section 2.5.1), von Mises
  limiter f_Y = min(Y0^2/(3 J2), 1) (section 2.6), density sum, continuity,
  momentum with artificial viscosity (section 3.1.2, 3.1.3), standard velocity
  gradient or the corrected one L C with C = M^-1, M = sum_b V_b (x_b - x_a) (x)
  grad_a W_ab (section 3.1.6; identity where M is singular), Hooke's law with
  Jaumann terms R S - S R (section 2.4), the Murnaghan equation of state
  (section 2.5.2: p = K0/n (eta^n - 1), K0 = rho0 c^2, the same tension cut-off,
  each particle's sound speed sqrt(K0/rho0 eta^(n-1)) averaged over the pair in Pi)
  when par[14] = 1, the artificial stress (section 3.1.4: (zeta_a + zeta_b) f^n in the
  momentum bracket, zeta = -eps_s T for a particle with negative pressure,
  f = W(r) / W(dmpd)) when par[10] > 0, the energy rate du/dt = 1/2 sum_b m_b
  (v_b - v_a) . (B g) with B the momentum bracket without artificial stress (section
  3.1.2) and the XSPH velocity v_a + xsph sum_b 2 m_b / (rho_a + rho_b) (v_b - v_a) W
  (section 3.1.5), and optionally a fixed damage field d
  (section 2.7): sigma_d = -p^ I + (1 - d) f_Y S, p^ = p for p >= 0 and (1 - d) p
  below, in the momentum equation only, and the Tillotson equation of state (section
  2.5.3) when par[14] = 2: the compressed form for rho >= rho0 or u <= E_iv, the
  expanded form for u >= E_cv, the two joined linearly in u between, an input u per
  particle, the sound speed sqrt(max(dp/drho + p / rho^2 dp/du, 0)) whose two partial
  derivatives autograd forms here with a graph of their own, so that the vector-Jacobian
  product reaches second derivatives of p (no hand derivation either).

Also the kick-drift-kick leapfrog used to drive the adjoint (the paper's own
integrators are the predictor-corrector and RK3 of section 3.4; the leapfrog
is the driver of the gradient workloads):

  F_0 = F(x_0, U_0),   U = (v, rho, S)
  U_{n+1/2} = U_n + dt/2 F_n          (S then limited by f_Y)
  x_{n+1}   = x_n + dt v_{n+1/2}
  F_{n+1}   = F(x_{n+1}, U_{n+1/2})
  U_{n+1}   = U_{n+1/2} + dt/2 F_{n+1}  (S then limited by f_Y)

Partner sets are recomputed by brute force (the C oracle) at every
evaluation; they are index sets and carry no derivative (every term of the
right-hand side vanishes with its first derivative at the support radius).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import native

SIGMA3 = 8.0 / math.pi
DT = torch.float64


def pairs_of(pos: torch.Tensor, h: float):
    """Ordered pairs (i target, j partner) by brute force on the detached positions."""
    row_ptr, col = native.neighbours(pos.detach().cpu().numpy(), h)
    counts = np.diff(row_ptr)
    i = torch.from_numpy(np.repeat(np.arange(counts.shape[0], dtype=np.int64), counts))
    j = torch.from_numpy(col.astype(np.int64))
    return i, j


def _mat(S6: torch.Tensor) -> torch.Tensor:
    """(6, n) -> (3, 3, n) symmetric."""
    xx, yy, zz, xy, xz, yz = S6
    return torch.stack([torch.stack([xx, xy, xz]), torch.stack([xy, yy, yz]),
                        torch.stack([xz, yz, zz])])


def _six(M: torch.Tensor) -> torch.Tensor:
    return torch.stack([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def yield_factor(S6: torch.Tensor, Y0) -> torch.Tensor:
    """f_Y = min(Y0^2 / (3 J2), 1), J2 = S:S/2 over the nine entries (section 2.6)."""
    J2 = 0.5 * (_mat(S6) ** 2).sum(dim=(0, 1))
    over = 3.0 * J2 > Y0 * Y0
    J2s = torch.where(over, J2, torch.ones_like(J2))
    return torch.where(over, Y0 * Y0 / (3.0 * J2s), torch.ones_like(J2))


def limit(S6: torch.Tensor, Y0) -> torch.Tensor:
    return yield_factor(S6, Y0) * S6


def correction_tensor(M: torch.Tensor) -> torch.Tensor:
    """C = M^-1 (3, 3, n) by the adjugate; the identity where det M <= 1e-12 (tr M / 3)^3."""
    m = M
    A = torch.stack([
        torch.stack([m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1], m[0, 2] * m[2, 1] - m[0, 1] * m[2, 2],
                     m[0, 1] * m[1, 2] - m[0, 2] * m[1, 1]]),
        torch.stack([m[1, 2] * m[2, 0] - m[1, 0] * m[2, 2], m[0, 0] * m[2, 2] - m[0, 2] * m[2, 0],
                     m[0, 2] * m[1, 0] - m[0, 0] * m[1, 2]]),
        torch.stack([m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0], m[0, 1] * m[2, 0] - m[0, 0] * m[2, 1],
                     m[0, 0] * m[1, 1] - m[0, 1] * m[1, 0]])])
    det = m[0, 0] * A[0, 0] + m[0, 1] * A[1, 0] + m[0, 2] * A[2, 0]
    t = (m[0, 0] + m[1, 1] + m[2, 2]) / 3.0
    ok = (det > 1e-12 * t * t * t) & torch.isfinite(det)
    eye = torch.eye(3, dtype=DT).unsqueeze(-1).expand_as(M)
    return torch.where(ok, A / torch.where(ok, det, torch.ones_like(det)), eye)


def tillotson(rho, u, par):
    """Tillotson pressure of section 2.5.3 per particle from eta = rho / rho0 and
    w = 1 + u / (E0 eta^2): the compressed form a rho u + b rho u / w + A (eta - 1)
    + B (eta - 1)^2 for rho >= rho0 or u <= E_iv, the expanded form a rho u +
    (b rho u / w + A (eta - 1) e^{-beta (rho0/rho - 1)}) e^{-alpha (rho0/rho - 1)^2} for
    u >= E_cv, and the straight line in u between the two in the remaining band."""
    rho0 = float(par[1])
    a, b, A, B, E0 = (float(par[k]) for k in (16, 17, 18, 19, 20))
    al, be, Eiv, Ecv = (float(par[k]) for k in (21, 22, 23, 24))
    eta = rho / rho0
    chi = eta - 1.0
    bw = b * rho * u / (1.0 + u / (E0 * eta * eta))
    p1 = a * rho * u + bw + A * chi + B * chi * chi
    z = rho0 / rho - 1.0
    p2 = a * rho * u + (bw + A * chi * torch.exp(-be * z)) * torch.exp(-al * z * z)
    t = (u - Eiv) / (Ecv - Eiv)
    mixed = (1.0 - t) * p1 + t * p2
    cold = (rho >= rho0) | (u <= Eiv)
    return torch.where(cold, p1, torch.where(u >= Ecv, p2, mixed))


def tillotson_pc(rho, u, par):
    """Pressure and sound speed of the Tillotson equation; the partial derivatives of p
    come from autograd on a graph of their own, kept so that c is differentiable."""
    r = rho if rho.requires_grad else rho.detach().clone().requires_grad_(True)
    e = u if u.requires_grad else u.detach().clone().requires_grad_(True)
    with torch.enable_grad():
        p = tillotson(r, e, par)
        pr, pu = torch.autograd.grad(p.sum(), [r, e], create_graph=True)
    c2 = pr + p / (r * r) * pu
    return p, torch.sqrt(torch.clamp(c2, min=0.0))


def rhs(pos, vel, rho, S6, m, par, mu=None, Y0=None, pairs=None, d=None, u=None):
    """Right-hand side of every particle.  ``par`` = {h, rho0, c, mu, Y0, alpha,
    beta, eps_v, rho_cut, correction}; ``mu``/``Y0`` may be tensors (differentiable)
    overriding par[3]/par[4]; ``d`` (n) a damage field held fixed.  Returns dict
    acc (3, n), drho, dS (6, n), rho_sum, L (3, 3, n) (L: the gradient that drives the
    stress rate, corrected when par[9] != 0); ``u`` (n) the specific internal energy, a
    tensor that may require grad, used by the Tillotson equation only."""
    h, rho0, c = float(par[0]), float(par[1]), float(par[2])
    alpha, beta, eps_v, rho_cut = float(par[5]), float(par[6]), float(par[7]), float(par[8])
    corr = len(par) > 9 and float(par[9]) != 0.0
    mu = float(par[3]) if mu is None else mu
    Y0 = float(par[4]) if Y0 is None else Y0
    n = rho.shape[0]
    if pairs is None:
        pairs = pairs_of(pos, h)
    i, j = pairs

    # prepass: pressure, limiter, stress
    eos = float(par[14]) if len(par) > 14 else 0.0
    if eos == 1.0:
        nM = float(par[15])
        K0 = rho0 * c * c
        eta = rho / rho0
        p = K0 / nM * (eta ** nM - 1.0)
        cs = torch.sqrt(K0 / rho0 * eta ** (nM - 1.0))
    elif eos == 0.0:
        p = c * c * (rho - rho0)
        cs = None
    elif eos == 2.0:
        if u is None:
            u = torch.zeros_like(rho)
        p, cs = tillotson_pc(rho, u, par)
    else:
        raise ValueError("equation of state %r" % eos)
    if rho_cut > 0 and eos != 2.0:
        p = torch.where(rho / rho0 < rho_cut, torch.zeros_like(p), p)
    f = yield_factor(S6, Y0)
    St = _mat(f * S6)
    eye = torch.eye(3, dtype=DT).unsqueeze(-1)
    if d is None:
        sig = St - p * eye
    else:
        keep = 1.0 - torch.as_tensor(np.asarray(d, dtype=np.float64))
        ph = torch.where(p >= 0, p, keep * p)
        sig = keep * St - ph * eye
    T = sig / (rho * rho)

    # pair terms
    rv = pos[:, i] - pos[:, j]
    r2 = (rv * rv).sum(0)
    r = torch.sqrt(r2)
    q = r / h
    inner = q < 0.5
    u = 1.0 - q
    W = SIGMA3 / h ** 3 * torch.where(inner, 6 * q ** 3 - 6 * q ** 2 + 1, 2 * u ** 3)
    dW = 6 * SIGMA3 / h ** 4 * torch.where(inner, 3 * q ** 2 - 2 * q, -(u * u))
    gW = dW / r * rv  # d W_ab / d x_a

    mj = m[j]
    rho_sum = m * (SIGMA3 / h ** 3) + torch.zeros(n, dtype=DT).index_add(0, i, mj * W)
    V = m / rho
    dv = vel[:, i] - vel[:, j]  # v_a - v_b
    cont = torch.zeros(n, dtype=DT).index_add(0, i, V[j] * (dv * gW).sum(0))
    drho = rho * cont
    Lp = -(V[j] * dv).unsqueeze(1) * gW.unsqueeze(0)  # (3, 3, P): (v_b - v_a)^a d_b W
    L = torch.zeros(3, 3, n, dtype=DT).index_add(2, i, Lp)
    w = (dv * rv).sum(0)
    nu = h * w / (r2 + eps_v * h * h)
    cbar = c if cs is None else 0.5 * (cs[i] + cs[j])
    Pi = torch.where(w < 0, (-alpha * cbar * nu + beta * nu * nu) / (0.5 * (rho[i] + rho[j])),
                     torch.zeros_like(w))
    B = T[:, :, i] + T[:, :, j] - Pi * eye
    dvb = -dv  # v_b - v_a
    up = 0.5 * mj * (dvb * (B * gW.unsqueeze(0)).sum(1)).sum(0)
    du = torch.zeros(n, dtype=DT).index_add(0, i, up)
    xsph = float(par[13]) if len(par) > 13 else 0.0
    xs = torch.zeros(3, n, dtype=DT).index_add(1, i, (2.0 * mj / (rho[i] + rho[j]) * W) * dvb)
    xv = vel + xsph * xs
    eps_s = float(par[10]) if len(par) > 10 else 0.0
    if eps_s > 0.0:
        n_s, dmpd = float(par[11]), float(par[12])
        qm = dmpd / h
        Wm = SIGMA3 / h ** 3 * (6 * qm ** 3 - 6 * qm ** 2 + 1 if qm < 0.5 else 2 * (1 - qm) ** 3)
        zeta = torch.where(p < 0, -eps_s * torch.ones_like(p), torch.zeros_like(p)) * T
        B = B + (zeta[:, :, i] + zeta[:, :, j]) * (W / Wm) ** n_s
    accp = mj * (B * gW.unsqueeze(0)).sum(1)
    acc = torch.zeros(3, n, dtype=DT).index_add(1, i, accp)

    # corrected gradient (the continuity sum above stays as printed)
    if corr:
        Mp = -(V[j] * rv).unsqueeze(1) * gW.unsqueeze(0)  # (x_b - x_a)^a d_g W
        M = torch.zeros(3, 3, n, dtype=DT).index_add(2, i, Mp)
        L = torch.einsum("agn,gbn->abn", L, correction_tensor(M))

    # postpass: Hooke + Jaumann
    Lt = L.transpose(0, 1)
    ed = 0.5 * (L + Lt)
    R = 0.5 * (L - Lt)
    tr = ed[0, 0] + ed[1, 1] + ed[2, 2]
    rot = torch.einsum("agn,gbn->abn", R, St) - torch.einsum("agn,gbn->abn", St, R)
    dSm = 2.0 * mu * (ed - tr / 3.0 * eye) + rot
    return dict(acc=acc, drho=drho, dS=_six(dSm), rho_sum=rho_sum, L=L, du=du, xv=xv)


def as_tensors(w):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    return t(w.pos), t(w.vel), t(w.rho), t(w.S), t(w.m), w.param_vector()


def rhs_vjp(w, cot: dict, pairs=None):
    """J^T y of one right-hand side: cotangents ``cot`` with keys acc (3, n), drho (n),
    dS (6, n), rho_sum (n) and optionally du (n) and xv (3, n).  Returns gradients pos,
    vel, rho, S (6, n), mu, Y0, and u (n; None unless the equation of state reads it)."""
    pos, vel, rho, S, m, par = as_tensors(w)
    u = torch.from_numpy(np.asarray(getattr(w, "u", None) if getattr(w, "u", None) is not None
                                    else np.zeros(w.n), dtype=np.float64)).requires_grad_(True)
    mu = torch.tensor(float(par[3]), dtype=DT, requires_grad=True)
    Y0 = torch.tensor(float(par[4]), dtype=DT, requires_grad=True)
    for t in (pos, vel, rho, S):
        t.requires_grad_(True)
    out = rhs(pos, vel, rho, S, m, par, mu=mu, Y0=Y0, pairs=pairs, d=getattr(w, "d", None), u=u)
    y = 0.0
    for k in ("acc", "drho", "dS", "rho_sum", "du", "xv"):
        if cot.get(k) is not None:
            y = y + (out[k] * torch.from_numpy(np.asarray(cot[k], dtype=np.float64))).sum()
    g = torch.autograd.grad(y, [pos, vel, rho, S, mu, Y0, u], allow_unused=True)
    names = ["pos", "vel", "rho", "S", "mu", "Y0", "u"]
    return {k: (v.detach().numpy() if v is not None else None) for k, v in zip(names, g)}


def leapfrog(pos, vel, rho, S6, m, par, steps: int, dt: float, mu=None, Y0=None, d=None):
    """Kick-drift-kick trajectory; returns the final (pos, vel, rho, S)."""
    Y0v = float(par[4]) if Y0 is None else Y0
    F = rhs(pos, vel, rho, S6, m, par, mu=mu, Y0=Y0, d=d)
    x, v, r, S = pos, vel, rho, S6
    for _ in range(steps):
        v = v + 0.5 * dt * F["acc"]
        r = r + 0.5 * dt * F["drho"]
        S = limit(S + 0.5 * dt * F["dS"], Y0v)
        x = x + dt * v
        F = rhs(x, v, r, S, m, par, mu=mu, Y0=Y0, d=d)
        v = v + 0.5 * dt * F["acc"]
        r = r + 0.5 * dt * F["drho"]
        S = limit(S + 0.5 * dt * F["dS"], Y0v)
    return x, v, r, S


def leapfrog_grad_all(w, steps: int, dt: float, cot: dict):
    """Gradients of the linear objective J = sum over fields f of <cot[f], f_final>
    (fields pos (3, n), vel (3, n), rho (n), S (6, n); missing ones count as zero)
    with respect to every initial field and to (mu, Y0).
    Returns dict J, pos, vel, rho, S (initial-state gradients), mu, Y0."""
    pos, vel, rho, S, m, par = as_tensors(w)
    for t in (pos, vel, rho, S):
        t.requires_grad_(True)
    mu = torch.tensor(float(par[3]), dtype=DT, requires_grad=True)
    Y0 = torch.tensor(float(par[4]), dtype=DT, requires_grad=True)
    final = dict(zip(("pos", "vel", "rho", "S"),
                     leapfrog(pos, vel, rho, S, m, par, steps, dt, mu=mu, Y0=Y0,
                              d=getattr(w, "d", None))))
    J = sum((torch.from_numpy(np.asarray(cot[k], dtype=np.float64)) * final[k]).sum()
            for k in final if k in cot)
    g = torch.autograd.grad(J, [pos, vel, rho, S, mu, Y0], allow_unused=True)
    like = (w.pos, w.vel, w.rho, w.S)
    out = {k: (g[i].detach().numpy() if g[i] is not None else np.zeros_like(like[i]))
           for i, k in enumerate(("pos", "vel", "rho", "S"))}
    out.update(J=float(J.detach()), mu=float(g[4]) if g[4] is not None else 0.0,
               Y0=float(g[5]) if g[5] is not None else 0.0)
    return out


def leapfrog_grad(w, steps: int, dt: float, objective: str = "ke", direction=None):
    """Gradients of a final-state objective with respect to (v0, mu, Y0).

    objective 'ke': J = sum_a m_a |v_a|^2 / 2;  'px'/'py'/'pz': J = sum_a m_a v_a^k;
    'dot': J = <direction, v_final> with ``direction`` (3, n).
    Returns dict J, v0 (3, n), mu, Y0.
    """
    pos, vel, rho, S, m, par = as_tensors(w)
    vel.requires_grad_(True)
    mu = torch.tensor(float(par[3]), dtype=DT, requires_grad=True)
    Y0 = torch.tensor(float(par[4]), dtype=DT, requires_grad=True)
    _, vT, _, _ = leapfrog(pos, vel, rho, S, m, par, steps, dt, mu=mu, Y0=Y0, d=getattr(w, "d", None))
    J = objective_value(vT, m, objective, direction)
    g = torch.autograd.grad(J, [vel, mu, Y0], allow_unused=True)
    z = lambda t, like: (t.detach().numpy() if t is not None else np.zeros_like(like))
    return dict(J=float(J.detach()), v0=z(g[0], w.vel), mu=float(g[1]) if g[1] is not None else 0.0,
                Y0=float(g[2]) if g[2] is not None else 0.0)


def objective_value(vT, m, objective: str, direction=None):
    if objective == "ke":
        return 0.5 * (m * (vT * vT).sum(0)).sum()
    if objective in ("px", "py", "pz"):
        k = "xyz".index(objective[1])
        return (m * vT[k]).sum()
    if objective == "dot":
        return (torch.from_numpy(np.asarray(direction, dtype=np.float64)) * vT).sum()
    raise ValueError(objective)


def leapfrog_value(w, steps: int, dt: float, objective: str = "ke", direction=None,
                   vel=None, mu=None, Y0=None) -> float:
    """Objective of the final state without gradients (for finite differences)."""
    pos, vel0, rho, S, m, par = as_tensors(w)
    if vel is not None:
        vel0 = torch.from_numpy(np.ascontiguousarray(vel, dtype=np.float64))
    with torch.no_grad():
        _, vT, _, _ = leapfrog(pos, vel0, rho, S, m, par, steps, dt,
                               mu=None if mu is None else float(mu),
                               Y0=None if Y0 is None else float(Y0), d=getattr(w, "d", None))
        return float(objective_value(vT, m, objective, direction))
