"""The seeded workloads the solver is tested and measured on.

Every generator takes a seed and returns a :class:`Problem`: the Hamiltonian,
the complex shifts z_k = eps_k + i*eta, and the right-hand sides (either unit
vectors e_j given by index, or dense complex vectors).  Sizes and value
distributions follow the workload recipes stated with each function.
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .csr import CSR, coo_to_csr
from .hubbard import hubbard_ring
from .lattices import diamond, simple_cubic


@dataclass
class Problem:
    name: str
    H: CSR
    z: np.ndarray  # complex128 [M]
    rhs_idx: Optional[np.ndarray] = None  # int64 [K] for unit-vector RHS e_j
    B: Optional[np.ndarray] = None  # complex128 [K, n] dense RHS (row j is b_j)
    tol: float = 1e-8
    max_iter: int = 3000
    extra: dict = field(default_factory=dict)

    @property
    def n_rhs(self) -> int:
        return len(self.rhs_idx) if self.rhs_idx is not None else self.B.shape[0]

    def rhs_dense(self) -> np.ndarray:
        """Right-hand sides as a dense complex [K, n] array."""
        if self.B is not None:
            return self.B
        b = np.zeros((len(self.rhs_idx), self.H.n), dtype=np.complex128)
        b[np.arange(len(self.rhs_idx)), self.rhs_idx] = 1.0
        return b


def shifts(lo: float, hi: float, m: int, eta: float) -> np.ndarray:
    return np.linspace(lo, hi, m) + 1j * eta


def config1_cubic(seed: int = 0, L: int = 16, n_shift: int = 64, disorder: float = 1.0) -> Problem:
    """Simple-cubic s-orbital lattice L^3 (periodic), hopping -1, on-site U[-disorder, disorder].

    64 shifts eps_k evenly spaced in [-7, 7] with eta = 0.01, RHS e_0,
    tolerance 1e-10, at most 3000 iterations; the output of interest is G_00.
    """
    rng = np.random.default_rng(seed)
    onsite = rng.uniform(-disorder, disorder, size=L ** 3) if disorder > 0 else np.zeros(L ** 3)
    H = simple_cubic(L, onsite)
    return Problem(f"cubic{L}", H, shifts(-7.0, 7.0, n_shift, 0.01), rhs_idx=np.array([0], dtype=np.int64),
                   tol=1e-10, max_iter=3000, extra=dict(L=L, onsite=onsite))


def config2_diamond(seed: int = 0, cells=(8, 8, 8), n_shift: int = 256, n_rhs: int = 256, eta: float = 0.005) -> Problem:
    """Diamond lattice, 4 orbitals per atom, displaced atoms and exp(-2(r-r0)) hopping.

    8x8x8 conventional cells = 4096 atoms = 16384 orbitals; 256 shifts with eps
    evenly spaced in [-12, 8] and eta = 0.005; RHS e_j for j = 0..n_rhs-1.
    """
    rng = np.random.default_rng(seed)
    H, geo = diamond(*cells, rng)
    return Problem(f"diamond{cells[0]}x{cells[1]}x{cells[2]}", H, shifts(-12.0, 8.0, n_shift, eta),
                   rhs_idx=np.arange(n_rhs, dtype=np.int64), tol=1e-8, max_iter=3000, extra=geo)


def config3_hubbard(seed: int = 0, L: int = 14, n_up: int = 7, n_dn: int = 7, n_shift: int = 128) -> Problem:
    """Extended Hubbard ring (t=1, U=4, V=1) in the fixed-(N_up, N_dn) sector.

    RHS is one seeded complex-normal vector normalised to unit 2-norm; 128 shifts
    eps in [-10, 20], eta = 0.05.
    """
    H = hubbard_ring(L, n_up, n_dn)
    z, b = config3_hubbard_rhs(seed, H.n, n_shift)
    return Problem(f"hubbard{L}_{n_up}u{n_dn}d", H, z, B=b[None, :],
                   tol=1e-8, max_iter=3000, extra=dict(L=L, n_up=n_up, n_dn=n_dn))


def config3_hubbard_rhs(seed: int, n: int, n_shift: int = 128):
    """The shifts and the seeded unit right-hand side of the Hubbard workload, without building
    its matrix (for the matrix-free operator): 128 shifts eps in [-10, 20], eta = 0.05; b complex
    normal, normalised to unit 2-norm."""
    rng = np.random.default_rng(seed)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    b /= np.linalg.norm(b)
    return shifts(-10.0, 20.0, n_shift, 0.05), b


def config4_diamond_small(seed: int = 0, cells=(2, 2, 1)) -> Problem:
    """Small diamond cells for the band-energy gradient checks (all orbitals as RHS).

    The shift list is left empty: the contour nodes are built by the caller.
    """
    rng = np.random.default_rng(seed)
    H, geo = diamond(*cells, rng)
    return Problem(f"diamond{cells[0]}x{cells[1]}x{cells[2]}", H, np.zeros(0, dtype=np.complex128),
                   rhs_idx=np.arange(H.n, dtype=np.int64), tol=1e-10, max_iter=5000, extra=geo)


def config5_batch(seed: int = 0, n_problems: int = 64, L_range=(24, 64), n_rhs: int = 32, n_shift: int = 512,
                  eta: float = 0.002):
    """Many disordered simple-cubic lattices of uneven size.

    L uniform in L_range (inclusive), disorder W uniform in {1, 4, 8} with on-site
    energies U[-W/2, W/2], hopping -1, n_rhs distinct seeded sites as RHS e_j,
    shifts eps in [-8, 8] with the given eta; tolerance 1e-8, at most 80,000 iterations (the
    slowest pairs at eta = 0.002 need about 66,000).
    """
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n_problems):
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        W = float(rng.choice([1.0, 4.0, 8.0]))
        onsite = rng.uniform(-W / 2, W / 2, size=L ** 3)
        H = simple_cubic(L, onsite)
        sites = np.sort(rng.choice(L ** 3, size=min(n_rhs, L ** 3), replace=False)).astype(np.int64)
        out.append(Problem(f"batch{q}_L{L}_W{W:g}", H, shifts(-8.0, 8.0, n_shift, eta), rhs_idx=sites,
                           tol=1e-8, max_iter=80000, extra=dict(L=L, W=W)))
    return out


def random_sparse_symmetric(n: int, density: float, rng: np.random.Generator, diag_scale: float = 1.0) -> CSR:
    """Random real-symmetric sparse matrix with a full diagonal (small test cases)."""
    mask = rng.random((n, n)) < density
    mask = np.triu(mask, 1)
    i, j = np.nonzero(mask)
    v = rng.uniform(-1.0, 1.0, size=len(i))
    d = rng.uniform(-diag_scale, diag_scale, size=n)
    rows = np.concatenate([i, j, np.arange(n)])
    cols = np.concatenate([j, i, np.arange(n)])
    vals = np.concatenate([v, v, d])
    return coo_to_csr(n, rows, cols, vals)
