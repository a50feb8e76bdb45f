"""CPU FP64 oracle of the SPH solid-body right-hand side (arXiv:1604.03290).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
in this package.  The product library (``paper_1604_03290_amd``) never does,
and the two share no code: the only common dependency is the seeded input
generator package ``workloads``, which holds none of the method's arithmetic.

  native    plain C (``sph_oracle.c``): brute-force partner sets, the
            right-hand side for any subset of targets, ball queries.
  autodiff  the same formulas in torch CPU float64 over an explicit pair
            list; reverse-mode AD gives the reference gradients, and the
            kick-drift-kick leapfrog that drives the gradient workloads.

Pins (tests/test_oracle_*.py) tie both to properties fixed by the paper and
by mathematics: kernel normalisation, lattice counts, conservation laws,
Hooke and rigid-rotation closed forms, limiter identities, finite
differences of the gradients.  The magnitude of the artificial-viscosity term
is pinned only through its symmetry, sign and scaling laws.
"""
from . import native  # noqa: F401
