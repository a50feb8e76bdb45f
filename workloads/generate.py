"""Seeded synthetic workloads (positions, velocities, densities, stresses, masses).

Every workload is a jittered cubic lattice (or a union of them) carrying the
material of the paper's aluminium impact test (section 4.3, impact cratering):
rho0 = 2700 kg/m^3, a linear equation of state with sound speed c = 5000 m/s,
shear modulus mu = 27 GPa, yield stress Y0 = 300 MPa, artificial viscosity
alpha = 0.5, beta = 0 (section 3.1.3, artificial viscosity).  Lengths are in
metres; the support radius of the cubic spline (the paper's h, section 3.1.1,
kernel function) is h = 2.4 lattice spacings, which gives about 56-61
interaction partners per interior particle.

Nothing here evaluates the method: no kernel, no SPH sums, no equation of
state.  Arrays are structure-of-arrays float64: positions (3, N), velocities
(3, N), deviatoric stress (6, N) in the order xx, yy, zz, xy, xz, yz, density
(N,), mass (N,).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 160403290
H_OVER_DX = 2.4

MATERIAL = dict(
    rho0=2700.0,
    c=5000.0,
    mu=2.7e10,
    Y0=3.0e8,
    alpha=0.5,
    beta=0.0,
    eps_v=0.01,
    rho_cut=0.0,
    correction=0.0,
    eps_s=0.0,   # artificial stress off (0.2 where used)
    n_s=4.0,     # its exponent
    xsph=0.0,    # XSPH off (0.5 where used)
    eos=0.0,     # 0 liquid, 1 Murnaghan, 2 Tillotson
    n_M=4.0,     # Murnaghan exponent (K0 = rho0 c^2)
    # Tillotson parameters of aluminium 6061 (section 4, impact cratering experiment)
    a_T=0.5, b_T=1.63, A_T=75.2e9, B_T=65e9, E0_T=5e6, alpha_T=5.0, beta_T=5.0,
    E_iv=3e6, E_cv=13.9e6,
)

# order of the scalar parameter vector shared by every consumer
PARAM_ORDER = ("h", "rho0", "c", "mu", "Y0", "alpha", "beta", "eps_v", "rho_cut", "correction",
               "eps_s", "n_s", "dmpd", "xsph", "eos", "n_M", "a_T", "b_T", "A_T", "B_T", "E0_T",
               "alpha_T", "beta_T", "E_iv", "E_cv")

CONFIG_NAMES = {
    0: "cube16_fp64_4096",
    1: "two_spheres_262144",
    2: "bullet_into_cube_2105344",
    3: "cube40_adjoint_64000",
    4: "nonuniform_8388608",
}


@dataclass
class Workload:
    name: str
    pos: np.ndarray
    vel: np.ndarray
    rho: np.ndarray
    S: np.ndarray
    m: np.ndarray
    h: float
    dx: float
    params: dict
    dt: float = 0.0
    steps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rho.shape[0])

    def param_vector(self) -> np.ndarray:
        return np.array([self.params[k] for k in PARAM_ORDER], dtype=np.float64)

    def box(self, margin: float | None = None):
        """Axis-aligned box holding every particle, padded by ``margin`` (default h)."""
        pad = self.h if margin is None else margin
        lo = self.pos.min(axis=1) - pad
        hi = self.pos.max(axis=1) + pad
        return lo, hi

    def copy(self) -> "Workload":
        w = Workload(
            self.name, self.pos.copy(), self.vel.copy(), self.rho.copy(), self.S.copy(),
            self.m.copy(), self.h, self.dx, dict(self.params), self.dt, self.steps, dict(self.meta),
        )
        for k in ("u", "d"):  # optional per-particle fields, set on some workloads
            if getattr(self, k, None) is not None:
                setattr(w, k, getattr(self, k).copy())
        return w

    def take(self, idx: np.ndarray) -> "Workload":
        """Sub-set of particles (same constants)."""
        idx = np.asarray(idx)
        return Workload(
            self.name + "_sub", np.ascontiguousarray(self.pos[:, idx]),
            np.ascontiguousarray(self.vel[:, idx]), np.ascontiguousarray(self.rho[idx]),
            np.ascontiguousarray(self.S[:, idx]), np.ascontiguousarray(self.m[idx]),
            self.h, self.dx, dict(self.params), self.dt, self.steps, dict(self.meta),
        )


def _params(h: float, **over) -> dict:
    p = dict(MATERIAL)
    p["h"] = float(h)
    p["dmpd"] = float(h) / H_OVER_DX  # mean particle distance of the initial lattice
    p.update(over)
    return p


def lattice_cube(n_side, dx: float, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Cell-centred cubic lattice points (i + 1/2) dx, x fastest; ``n_side`` int or (nx, ny, nz)."""
    if np.isscalar(n_side):
        nx = ny = nz = int(n_side)
    else:
        nx, ny, nz = (int(v) for v in n_side)
    ix = (np.arange(nx) + 0.5) * dx + origin[0]
    iy = (np.arange(ny) + 0.5) * dx + origin[1]
    iz = (np.arange(nz) + 0.5) * dx + origin[2]
    z, y, x = np.meshgrid(iz, iy, ix, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()]))


def _jitter(pos: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    return pos + rng.normal(0.0, sigma, size=pos.shape)


def random_state(n: int, rng: np.random.Generator, rho0: float, c: float, rho_scale=1.0):
    """Velocities ~ N(0, (0.01 c)^2) per component; rho = rho0 (1 + 0.01 xi) * rho_scale;
    deviatoric stress: six independent N(0, s^2), s = 1e-3 rho0 c^2, with the mean of
    the three diagonal entries removed so that it is traceless."""
    vel = rng.normal(0.0, 0.01 * c, size=(3, n))
    rho = rho0 * rho_scale * (1.0 + 0.01 * rng.normal(0.0, 1.0, size=n))
    s = 1e-3 * rho0 * c * c
    S = rng.normal(0.0, s, size=(6, n))
    tr3 = (S[0] + S[1] + S[2]) / 3.0
    S[0] -= tr3
    S[1] -= tr3
    S[2] -= tr3
    return vel, rho, S


def cube(n_side: int, dx: float, seed: int, jitter: float = 0.05, state: str = "random",
         name: str | None = None, shuffle: bool = False, h_over_dx: float = H_OVER_DX,
         **param_over) -> Workload:
    """Jittered cubic block of n_side^3 particles with spacing dx."""
    rng = np.random.default_rng(seed)
    pos = lattice_cube(n_side, dx)
    n = pos.shape[1]
    if jitter > 0:
        pos = _jitter(pos, jitter * dx, rng)
    p = _params(h_over_dx * dx, **param_over)
    if state == "random":
        vel, rho, S = random_state(n, rng, p["rho0"], p["c"])
    elif state == "rest":
        vel = np.zeros((3, n))
        rho = np.full(n, p["rho0"])
        S = np.zeros((6, n))
    else:
        raise ValueError(state)
    m = np.full(n, p["rho0"] * dx ** 3)
    w = Workload(name or f"cube{n_side}", np.ascontiguousarray(pos), vel, rho, S, m,
                 p["h"], dx, p, dt=0.2 * dx / p["c"])
    if shuffle:
        order = rng.permutation(n)
        w = w.take(order)
        w.name = name or f"cube{n_side}_shuffled"
    return w


def _ball_lattice(n_keep: int, dx: float, r_min: float = 0.0) -> np.ndarray:
    """The n_keep cell-centred lattice points nearest the origin with radius >= r_min
    (ties broken by lexicographic lattice index); returns (3, n_keep) centred at 0."""
    # radius needed, with 10 % slack, from the volume per point
    if r_min <= 0:
        r_need = (3.0 * n_keep / (4.0 * math.pi)) ** (1.0 / 3.0) * dx * 1.1 + 2 * dx
    else:
        r_need = ((r_min / dx) ** 3 + 3.0 * n_keep / (4.0 * math.pi)) ** (1.0 / 3.0) * dx * 1.05 + 2 * dx
    M = int(math.ceil(r_need / dx))
    k = np.arange(-M, M, dtype=np.int64) * 2 + 1  # 2 i + 1: exact integer radii
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    r2 = (kx * kx + ky * ky + kz * kz).ravel()  # (2r/dx)^2, exact
    sel = np.nonzero(r2 >= int(math.floor((2.0 * r_min / dx) ** 2)))[0] if r_min > 0 else None
    if sel is not None:
        # strictly: r >= r_min, evaluated in float after the integer pre-filter
        rr = np.sqrt(r2[sel].astype(np.float64)) * (0.5 * dx)
        sel = sel[rr >= r_min]
        order = sel[np.argsort(r2[sel], kind="stable")]
    else:
        order = np.argsort(r2, kind="stable")
    if order.shape[0] < n_keep:
        raise RuntimeError("lattice too small")
    keep = order[:n_keep]
    pts = np.stack([kx.ravel()[keep], ky.ravel()[keep], kz.ravel()[keep]]).astype(np.float64) * (0.5 * dx)
    return np.ascontiguousarray(pts)


def _config0(seed):
    return cube(16, 1.0 / 16.0, seed, name=CONFIG_NAMES[0])


def _config1(seed):
    rng = np.random.default_rng(seed)
    n_half = 131072
    dx = (4.0 * math.pi / 3.0 / n_half) ** (1.0 / 3.0)
    ball = _ball_lattice(n_half, dx)
    sep = math.sqrt((2.0 + dx) ** 2 - 0.25)
    a = _jitter(ball, 0.05 * dx, rng) + np.array([[-0.5 * sep], [-0.25], [0.0]])
    b = _jitter(ball, 0.05 * dx, rng) + np.array([[0.5 * sep], [0.25], [0.0]])
    pos = np.ascontiguousarray(np.concatenate([a, b], axis=1))
    n = pos.shape[1]
    p = _params(H_OVER_DX * dx)
    vel = np.zeros((3, n))
    vel[0, :n_half] = 0.025 * p["c"]
    vel[0, n_half:] = -0.025 * p["c"]
    rho = np.full(n, p["rho0"])
    S = np.zeros((6, n))
    m = np.full(n, p["rho0"] * dx ** 3)
    return Workload(CONFIG_NAMES[1], pos, vel, rho, S, m, p["h"], dx, p,
                    dt=0.2 * dx / p["c"], steps=10, meta=dict(n_sphere=n_half))


def _config2(seed, state="impact"):
    rng = np.random.default_rng(seed)
    dx = 1.0 / 128.0
    target = _jitter(lattice_cube(128, dx), 0.05 * dx, rng)
    # projectile: lattice columns inside a radius-0.1 cylinder about (0.5, 0.5),
    # layers from z = 1 + dx upwards, 8192 points nearest the bottom / axis
    k = (np.arange(128) + 0.5) * dx
    yy, xx = np.meshgrid(k, k, indexing="ij")
    rr2 = ((xx - 0.5) ** 2 + (yy - 0.5) ** 2).ravel()
    col = np.nonzero(rr2 <= 0.1 ** 2)[0]
    col = col[np.argsort(rr2[col], kind="stable")]
    n_proj = 8192
    layers = -(-n_proj // col.shape[0])
    pts = []
    for L in range(layers):
        take = col[: min(col.shape[0], n_proj - L * col.shape[0])]
        z = 1.0 + dx + L * dx
        pts.append(np.stack([xx.ravel()[take], yy.ravel()[take], np.full(take.shape[0], z)]))
    proj = _jitter(np.concatenate(pts, axis=1), 0.05 * dx, rng)
    pos = np.ascontiguousarray(np.concatenate([target, proj], axis=1))
    n = pos.shape[1]
    p = _params(H_OVER_DX * dx)
    if state == "impact":
        vel = np.zeros((3, n))
        vel[2, target.shape[1]:] = -0.2 * p["c"]
        rho = np.full(n, p["rho0"])
        S = np.zeros((6, n))
    elif state == "random":
        vel, rho, S = random_state(n, rng, p["rho0"], p["c"])
    else:
        raise ValueError(state)
    m = np.full(n, p["rho0"] * dx ** 3)
    return Workload(CONFIG_NAMES[2] + ("" if state == "impact" else "_random"), pos, vel, rho, S, m,
                    p["h"], dx, p, dt=0.2 * dx / p["c"], steps=1, meta=dict(n_target=target.shape[1]))


def _config3(seed):
    w = cube(40, 1.0 / 16.0, seed, name=CONFIG_NAMES[3])
    w.steps = 20
    return w


def _config4(seed):
    rng = np.random.default_rng(seed)
    nA, nB, nS = 4194304, 3145728, 1048576
    dx = (4.0 * math.pi / 3.0 / nB) ** (1.0 / 3.0)  # sphere B: radius 1
    h = H_OVER_DX * dx
    sA, sS = 0.615 * dx, 1.39 * dx
    rA = (3.0 * nA / (4.0 * math.pi)) ** (1.0 / 3.0) * sA
    rB = 1.0
    A = _jitter(_ball_lattice(nA, sA), 0.05 * sA, rng) + np.array([[-(rA + h)], [0.0], [0.0]])
    B = _jitter(_ball_lattice(nB, dx), 0.05 * dx, rng) + np.array([[rB + h], [0.0], [0.0]])
    mid = 0.5 * ((-(rA + h) - rA) + (rB + h + rB))
    Sh = _jitter(_ball_lattice(nS, sS, r_min=2.0), 0.05 * sS, rng) + np.array([[mid], [0.0], [0.0]])
    pos = np.ascontiguousarray(np.concatenate([A, B, Sh], axis=1))
    n = pos.shape[1]
    p = _params(h)
    scale = np.concatenate([np.full(nA, (dx / sA) ** 3), np.full(nB, 1.0), np.full(nS, (dx / sS) ** 3)])
    vel, rho, S = random_state(n, rng, p["rho0"], p["c"])
    rho = rho * scale
    m = np.full(n, p["rho0"] * dx ** 3)
    return Workload(CONFIG_NAMES[4], pos, vel, rho, S, m, h, dx, p, dt=0.2 * dx / p["c"], steps=1,
                    meta=dict(nA=nA, nB=nB, nS=nS, spacing=(sA, dx, sS)))


def config(k: int, seed: int | None = None, **kw) -> Workload:
    """Workload k (0..4) with the default seed SEED_BASE + k."""
    seed = SEED_BASE + k if seed is None else seed
    f = {0: _config0, 1: _config1, 2: _config2, 3: _config3, 4: _config4}[k]
    return f(seed, **kw)


def two_particles(xa, xb, va=(0, 0, 0), vb=(0, 0, 0), rho=(2700.0, 2700.0), S=None, m=(1.0, 1.0),
                  h=1.0, **param_over) -> Workload:
    """Two-particle set for closed-form checks."""
    pos = np.ascontiguousarray(np.array([xa, xb], dtype=np.float64).T)
    vel = np.ascontiguousarray(np.array([va, vb], dtype=np.float64).T)
    Sarr = np.zeros((6, 2)) if S is None else np.ascontiguousarray(np.array(S, dtype=np.float64).T)
    p = _params(h, **param_over)
    return Workload("pair", pos, vel, np.array(rho, dtype=np.float64), Sarr,
                    np.array(m, dtype=np.float64), float(h), float(h) / H_OVER_DX, p)


def flaws(n: int, volume: float, k_w: float, m_w: float, seed: int):
    """Activation threshold strains of the damage model's preprocessing (the damage model
    of section 3): flaw j = 1, 2, ... goes to a particle drawn uniformly at random with
    threshold (j / (k_w volume))^(1 / m_w) (Weibull parameters k_w, m_w), until every
    particle holds at least one.  Returns (flaw_ptr int64 [n + 1], flaw_eps [total]), each
    particle's thresholds ascending."""
    rng = np.random.default_rng(seed)
    seen = np.zeros(n, dtype=bool)
    remaining = n
    chunks = []
    while True:
        chunk = rng.integers(0, n, max(n, 64))
        pos = np.nonzero(~seen[chunk])[0]
        new, first = np.unique(chunk[pos], return_index=True)
        if new.size == remaining:  # the last particle without a flaw gets one here
            chunks.append(chunk[: pos[first].max() + 1])
            break
        seen[new] = True
        remaining -= new.size
        chunks.append(chunk)
    owner = np.concatenate(chunks)
    total = owner.size
    j = np.arange(1, total + 1, dtype=np.float64)
    eps = (j / (k_w * volume)) ** (1.0 / m_w)
    order = np.argsort(owner, kind="stable")
    counts = np.bincount(owner, minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    return ptr, np.ascontiguousarray(eps[order])


def subsample(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct particle indices drawn uniformly without replacement, ascending."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
