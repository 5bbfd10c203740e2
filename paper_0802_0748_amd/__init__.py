"""Shifted-COCG Green's-function solver for MI355X (gfx950).

The compute path is libscocg.so (hand-written HIP kernels behind a C ABI,
declared in include/scocg.h); this package is its Python binding, with
PyTorch used for device memory, streams and autograd.
"""

from .api import (Hamiltonian, Tape, backward, contour, csr_validate, density_matrix_energy, greens_diag, greens_diag_noalloc,
                  greens_diag_batched, greens_diag_waves, greens_proj, ground_state, hubbard_fermion_op,
                  krylov_greens_diag, krylov_greens_vec, last_switches, last_timing, options, set_profiling, shifted_cocg_solve)

__all__ = [
    "Hamiltonian",
    "Tape",
    "backward",
    "contour",
    "csr_validate",
    "density_matrix_energy",
    "greens_diag",
    "greens_diag_batched",
    "greens_diag_noalloc",
    "greens_diag_waves",
    "greens_proj",
    "ground_state",
    "hubbard_fermion_op",
    "krylov_greens_diag",
    "krylov_greens_vec",
    "last_switches",
    "last_timing",
    "options",
    "set_profiling",
    "shifted_cocg_solve",
]
