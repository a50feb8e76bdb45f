"""MI355X (gfx950) implementation of the SPH solid-body right-hand side of
Schaefer et al. (2016), arXiv:1604.03290: cell-list partner search, density
sum, continuity, momentum with the full stress tensor and artificial
viscosity, velocity gradient, Hooke's law with Jaumann rotation terms, von
Mises limiter; its hand-written adjoint; a checkpointed leapfrog.

The computation lives in libsph.so (HIP kernels behind the C ABI of
include/sph.h).  This package only binds it to torch tensors.
"""
from . import _lib  # noqa: F401
from .api import (  # noqa: F401
    CellGrid,
    ParticleState,
    SphRhs,
    sph_build_cells,
    sph_build_pairs,
    sph_gravity,
    sph_leapfrog,
    sph_leapfrog_adjoint,
    sph_neighbours,
    sph_rhs,
    sph_rhs_adjoint,
    sph_rhs_noalloc,
    workspace,
    workspace_status,
)
from ._lib import SPH_FP32_COMP, SPH_FP64, SphError  # noqa: F401

build_cells = sph_build_cells
build_pairs = sph_build_pairs
neighbours = sph_neighbours
rhs = sph_rhs
rhs_adjoint = sph_rhs_adjoint
leapfrog = sph_leapfrog
leapfrog_adjoint = sph_leapfrog_adjoint
