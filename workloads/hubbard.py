"""One-dimensional extended Hubbard ring in the occupation-number basis.

Stands in for the many-electron workload of Sec. 4.2 (an extended Hubbard model
whose S_z sector Hamiltonian is a huge sparse matrix, Sec. 2.2).  The model here
is the single-orbital ring

    H = -t sum_{i,s} (c+_{i,s} c_{i+1,s} + h.c.) + U sum_i n_{i,up} n_{i,dn}
        + V sum_i n_i n_{i+1},        n_i = n_{i,up} + n_{i,dn},

on L sites with periodic boundary, restricted to fixed (N_up, N_dn).

Basis: each spin species is a bit string of L bits (bit i = site i occupied)
with N_s bits set, listed in increasing integer order; the sector state is
index = i_up * D_dn + i_dn.  Fermion signs follow the Jordan-Wigner ordering
with all up-spin modes before all down-spin modes, so a hop of one species only
sees that species' electrons between the two sites.  An interior bond (i, i+1)
has sign +1; the ring-closing bond (L-1, 0) has sign (-1)^(N_s - 1).
"""

import numpy as np

from .csr import CSR


def sector_basis(L: int, n: int) -> np.ndarray:
    """All L-bit integers with n bits set, ascending."""
    from itertools import combinations

    states = [sum(1 << i for i in c) for c in combinations(range(L), n)]
    return np.array(sorted(states), dtype=np.int64)


def _popcount(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    y = x.copy()
    while np.any(y):
        c += y & 1
        y >>= 1
    return c


def _rot(x: np.ndarray, L: int) -> np.ndarray:
    """Bit i of the result is bit (i+1) mod L of x (the right neighbour's occupation)."""
    return ((x >> 1) | ((x & 1) << (L - 1))) & ((1 << L) - 1)


def species_hopping(L: int, n: int, t: float):
    """Hopping matrix of one species as (row_ptr, col, val), columns sorted."""
    states = sector_basis(L, n)
    lookup = {int(s): k for k, s in enumerate(states)}
    bonds = [(i, (i + 1) % L) for i in range(L)]
    ptr = [0]
    cols = []
    vals = []
    for s in states:
        row = {}
        for i, j in bonds:
            bi = (int(s) >> i) & 1
            bj = (int(s) >> j) & 1
            if bi == bj:
                continue
            ns = int(s) ^ ((1 << i) | (1 << j))
            sign = 1.0
            if (i, j) == (L - 1, 0):
                sign = (-1.0) ** (n - 1)
            k = lookup[ns]
            row[k] = row.get(k, 0.0) - t * sign
        for k in sorted(row):
            cols.append(k)
            vals.append(row[k])
        ptr.append(len(cols))
    return np.array(ptr, dtype=np.int64), np.array(cols, dtype=np.int64), np.array(vals, dtype=np.float64)


def hubbard_diagonal(L: int, up: np.ndarray, dn: np.ndarray, U: float, V: float) -> np.ndarray:
    """Diagonal energies for every (i_up, i_dn) pair, shape [D_up, D_dn]."""
    u = up[:, None]
    d = dn[None, :]
    onsite = _popcount(u & d)
    ru = _rot(u, L)
    rd = _rot(d, L)
    inter = _popcount(u & ru) + _popcount(d & rd) + _popcount(u & rd) + _popcount(d & ru)
    return U * onsite + V * inter


def hubbard_ring(L: int, n_up: int, n_dn: int, t: float = 1.0, U: float = 4.0, V: float = 1.0) -> CSR:
    """Sector Hamiltonian as CSR with int64 indices; the diagonal is always stored.

    The matrix has the Kronecker-sum structure T_up (x) 1 + 1 (x) T_dn + D, which
    is used here only to assemble the rows quickly.
    """
    if L < 3:
        raise ValueError("ring needs at least 3 sites")
    up = sector_basis(L, n_up)
    dn = sector_basis(L, n_dn)
    Du, Dd = len(up), len(dn)
    diag = hubbard_diagonal(L, up, dn, U, V).astype(np.float64)
    up_ptr, up_col, up_val = species_hopping(L, n_up, t)
    dn_ptr, dn_col, dn_val = species_hopping(L, n_dn, t)

    # Down-spin block row with the diagonal merged in (marker position kept).
    dn_len = np.diff(dn_ptr) + 1
    mid_ptr = np.concatenate([[0], np.cumsum(dn_len)])
    mid_col = np.empty(mid_ptr[-1], dtype=np.int64)
    mid_val = np.empty(mid_ptr[-1], dtype=np.float64)
    mid_isdiag = np.zeros(mid_ptr[-1], dtype=bool)
    for r in range(Dd):
        c = np.concatenate([dn_col[dn_ptr[r]:dn_ptr[r + 1]], [r]])
        v = np.concatenate([dn_val[dn_ptr[r]:dn_ptr[r + 1]], [0.0]])
        isd = np.zeros(len(c), dtype=bool)
        isd[-1] = True
        o = np.argsort(c, kind="stable")
        s = slice(mid_ptr[r], mid_ptr[r + 1])
        mid_col[s] = c[o]
        mid_val[s] = v[o]
        mid_isdiag[s] = isd[o]
    mid_rows = np.repeat(np.arange(Dd), dn_len)
    diag_pos = np.nonzero(mid_isdiag)[0]

    n = Du * Dd
    up_len = np.diff(up_ptr)
    row_len = up_len[:, None] + dn_len[None, :]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(row_len.ravel(), out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int64)
    val = np.empty(nnz, dtype=np.float64)

    ids = np.arange(Dd, dtype=np.int64)
    for iu in range(Du):
        ju = up_col[up_ptr[iu]:up_ptr[iu + 1]]
        tu = up_val[up_ptr[iu]:up_ptr[iu + 1]]
        lower = ju < iu
        ju_l, tu_l = ju[lower], tu[lower]
        ju_u, tu_u = ju[~lower], tu[~lower]
        kl = len(ju_l)
        start = row_ptr[iu * Dd:(iu + 1) * Dd]
        for m in range(kl):
            p = start + m
            col[p] = ju_l[m] * Dd + ids
            val[p] = tu_l[m]
        # mid block: positions start[id] + kl + offset within the merged down row
        pos = start[mid_rows] + kl + (np.arange(len(mid_col)) - mid_ptr[mid_rows])
        col[pos] = iu * Dd + mid_col
        mv = mid_val.copy()
        mv[diag_pos] = diag[iu, :]
        val[pos] = mv
        for m in range(len(ju_u)):
            p = start + kl + dn_len + m
            col[p] = ju_u[m] * Dd + ids
            val[p] = tu_u[m]
    return CSR(n, row_ptr, col, val)
