"""TEST INFRASTRUCTURE: oracle of the damage growth rate of the Grady-Kipp model
(section 2.7 and the damage model of section 3), per particle.  Only the test-suite
uses it; it shares no code with the HIP library.

  sigma_d          the damaged stress of the C oracle's prepass (-p^ I + (1 - d) f_Y S)
  sigma_max        the largest principal stress (LAPACK eigenvalues of sigma_d)
  epsilon          sigma_max / ((1 - d) E), E = 9 K mu / (3 K + mu)
  n_act            flaws of the particle whose activation threshold lies below epsilon
  d(d^(1/3))/dt    n_act c_g / R_s, c_g = 0.4 sqrt((K + 4/3 (1 - d) mu) / rho),
                   zero once d has reached the limiter d_max = n_act / n_tot

Readings: the printed crack speed 0.4 (1/rho) sqrt(K0 + 4/3 (1 - d) mu) is not a
velocity; 0.4 times the longitudinal wave speed is sqrt((K0 + 4/3 (1 - d) mu) / rho),
as the text says.  R_s is the radius of the particle's own volume,
4/3 pi R_s^3 = m / rho.  K is rho0 c^2 for the liquid and Murnaghan equations and A_T
for Tillotson.  A fully damaged particle (d = 1) has every flaw active.  The limiter
acts on the rate: growth stops while d >= n_act / n_tot (n_tot the particle's flaw
count), so an integrator never carries d past it.
"""
import numpy as np

from . import native
from workloads.generate import PARAM_ORDER

_I = {k: i for i, k in enumerate(PARAM_ORDER)}


def bulk_modulus(par) -> float:
    par = np.asarray(par, dtype=np.float64)
    if par[_I["eos"]] == 2.0:
        return float(par[_I["A_T"]])
    return float(par[_I["rho0"]] * par[_I["c"]] ** 2)


def young_modulus(K: float, mu: float) -> float:
    return 9.0 * K * mu / (3.0 * K + mu)


def principal_max(sigma6: np.ndarray) -> np.ndarray:
    """Largest eigenvalue of each symmetric stress (6, n: xx yy zz xy xz yz)."""
    s = sigma6
    M = np.empty((s.shape[1], 3, 3))
    M[:, 0, 0], M[:, 1, 1], M[:, 2, 2] = s[0], s[1], s[2]
    M[:, 0, 1] = M[:, 1, 0] = s[3]
    M[:, 0, 2] = M[:, 2, 0] = s[4]
    M[:, 1, 2] = M[:, 2, 1] = s[5]
    return np.linalg.eigvalsh(M)[:, -1]


def rates(rho, S, m, par, flaw_ptr, flaw_eps, u=None, d=None):
    """(d(d^(1/3))/dt, n_act, epsilon) of every particle."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape[0]
    dd = np.zeros(n) if d is None else np.asarray(d, dtype=np.float64)
    pre = native.prepass2(rho, S, par, u, d)
    mu = float(np.asarray(par)[_I["mu"]])
    K = bulk_modulus(par)
    E = young_modulus(K, mu)
    smax = principal_max(pre["sigma"])
    with np.errstate(divide="ignore", invalid="ignore"):
        eps = np.where(dd < 1.0, smax / ((1.0 - dd) * E), np.inf)
    nact = np.zeros(n, dtype=np.int64)
    for a in range(n):
        f = flaw_eps[flaw_ptr[a]:flaw_ptr[a + 1]]
        nact[a] = int(np.searchsorted(f, eps[a], side="left"))
    cg = 0.4 * np.sqrt((K + 4.0 / 3.0 * (1.0 - dd) * mu) / rho)
    Rs = np.cbrt(3.0 * np.asarray(m, dtype=np.float64) / (4.0 * np.pi * rho))
    ntot = np.diff(np.asarray(flaw_ptr, dtype=np.int64))
    grow = dd * ntot < nact
    return np.where(grow, nact * cg / Rs, 0.0), nact, eps
