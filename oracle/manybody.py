"""Many-electron reference (plain FP64 CPU): ground state and single-particle excitations of
the Hubbard ring's S_z sectors, for Sec. 2.2 (ground state by Lanczos and CG inverse
iteration, then the excitation spectra of Sec. 4.2).

TEST INFRASTRUCTURE ONLY: the test suite uses this module.  It shares no code with the GPU
library.

Conventions (those of the sector matrices in workloads/hubbard.py): a sector (L, N_up, N_dn)
has the basis |s_up, s_dn> with s_s an L-bit pattern (bit i = site i occupied) listed in
increasing integer order, index i_up * D_dn + i_dn; the state is the product of creation
operators in Jordan-Wigner order, all up-spin modes (sites ascending) before all down-spin
modes.  So c_{i,s} and c+_{i,s} act with the sign (-1)^(number of occupied modes before
(i, s) in that order).
"""

import numpy as np


def basis(L: int, n: int) -> np.ndarray:
    """The L-bit patterns with n bits set, ascending."""
    return np.array([s for s in range(1 << L) if bin(s).count("1") == n], dtype=np.int64)


def fermion_op(L: int, n_up: int, n_dn: int, site: int, spin: int, create: bool, x: np.ndarray):
    """c_{site,spin} x (create=False) or c+_{site,spin} x (create=True) for x in sector
    (L, n_up, n_dn); returns (y, (n_up', n_dn')) with y in the target sector.  spin 0 = up."""
    up, dn = basis(L, n_up), basis(L, n_dn)
    d = 1 if create else -1
    tu, td = (n_up + d, n_dn) if spin == 0 else (n_up, n_dn + d)
    up_t, dn_t = basis(L, tu), basis(L, td)
    rank_up = {int(s): k for k, s in enumerate(up_t)}
    rank_dn = {int(s): k for k, s in enumerate(dn_t)}
    y = np.zeros(len(up_t) * len(dn_t), dtype=x.dtype)
    bit = 1 << site
    for iu, su in enumerate(up):
        for idn, sd in enumerate(dn):
            s = int(su) if spin == 0 else int(sd)
            occupied = bool(s & bit)
            if occupied == create:
                continue
            before = bin(s & (bit - 1)).count("1") + (0 if spin == 0 else n_up)
            sign = -1.0 if before % 2 else 1.0
            if spin == 0:
                k = rank_up[int(su) ^ bit] * len(dn_t) + idn
            else:
                k = iu * len(dn_t) + rank_dn[int(sd) ^ bit]
            y[k] += sign * x[iu * len(dn) + idn]
    return y, (tu, td)


def ground_state(Hdense: np.ndarray):
    """Lowest eigenpair (E0, psi0) of a sector matrix by dense diagonalization; psi0 has a
    positive largest component (the sign is otherwise free)."""
    e, v = np.linalg.eigh(Hdense)
    psi = v[:, 0]
    if psi[np.argmax(np.abs(psi))] < 0:
        psi = -psi
    return float(e[0]), psi, float(e[1])


def projected_resolvent(Hdense: np.ndarray, b: np.ndarray, z):
    """<b|(z - H)^{-1}|b> (bilinear, b real) for each z, by dense solves."""
    n = len(b)
    return np.array([b @ np.linalg.solve(zk * np.eye(n) - Hdense, b.astype(complex)) for zk in np.atleast_1d(z)])
