"""Seeded synthetic inputs for the shifted-COCG Green's-function solver.

This package builds the *inputs* only: sparse real-symmetric Hamiltonians in
CSR form, shift lists z_k = eps_k + i*eta and right-hand sides.  It contains
none of the solver's arithmetic, so both the CPU oracle and the GPU path can
consume what it produces without sharing any method code.

The Hamiltonians stand in for the paper's workloads (tight-binding solids,
Sec. 2.1 and 4.1; the extended Hubbard model, Sec. 4.2), whose parameter sets
are not reproduced here.
"""

from .csr import CSR, coo_to_csr
from .lattices import simple_cubic, diamond
from .hubbard import hubbard_ring, sector_basis
from .configs import (
    Problem,
    config1_cubic,
    config2_diamond,
    config3_hubbard,
    config3_hubbard_rhs,
    config4_diamond_small,
    config5_batch,
    random_sparse_symmetric,
)

__all__ = [
    "CSR",
    "coo_to_csr",
    "simple_cubic",
    "diamond",
    "hubbard_ring",
    "sector_basis",
    "Problem",
    "config1_cubic",
    "config2_diamond",
    "config3_hubbard",
    "config3_hubbard_rhs",
    "config4_diamond_small",
    "config5_batch",
    "random_sparse_symmetric",
]
