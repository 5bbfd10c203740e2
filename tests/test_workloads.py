"""Checks of the seeded input generators (shapes, symmetry, and an independent
brute-force construction of the Hubbard sector Hamiltonian)."""

import numpy as np
import pytest

from workloads import (config1_cubic, config2_diamond, config3_hubbard, config4_diamond_small, config5_batch,
                       hubbard_ring, sector_basis)


def _sorted_unique_rows(H):
    for i in range(H.n):
        c = H.col[H.row_ptr[i]:H.row_ptr[i + 1]]
        if np.any(np.diff(c) <= 0):
            return False
    return True


def test_config1_shape():
    p = config1_cubic()
    assert p.H.n == 4096 and p.H.nnz == 28672
    assert len(p.z) == 64 and np.allclose(p.z.imag, 0.01)
    assert np.isclose(p.z.real[0], -7) and np.isclose(p.z.real[-1], 7)
    A = p.H.to_scipy()
    assert abs(A - A.T).max() == 0
    assert _sorted_unique_rows(p.H)


def test_config2_shape():
    p = config2_diamond()
    assert p.H.n == 16384 and p.H.nnz == 278528
    assert np.all(np.diff(p.H.row_ptr) == 17)
    assert len(p.z) == 256 and p.n_rhs == 256
    A = p.H.to_scipy()
    assert abs(A - A.T).max() == 0
    d = p.H.diagonal()
    assert np.array_equal(d[:4], [-5, 1, 1, 1])


def test_config4_small_cells():
    p = config4_diamond_small()
    assert p.H.n == 128
    assert np.all(np.diff(p.H.row_ptr) == 17)
    p = config4_diamond_small(cells=(2, 2, 2))
    assert p.H.n == 256


def test_config5_sizes():
    ps = config5_batch(n_problems=4, L_range=(3, 5), n_rhs=4, n_shift=8)
    for p in ps:
        L = p.extra["L"]
        assert p.H.n == L ** 3 and 3 <= L <= 5
        assert len(np.unique(p.rhs_idx)) == 4


def _fock_hamiltonian(L, t, U, V):
    """Brute-force Fock-space Hamiltonian: modes 0..L-1 spin up, L..2L-1 spin down,
    basis state s = product of c+_m over set bits in increasing m acting on |0>."""
    dim = 1 << (2 * L)
    H = np.zeros((dim, dim))

    def apply_c(m, s):
        if not (s >> m) & 1:
            return None, 0
        sign = (-1) ** bin(s & ((1 << m) - 1)).count("1")
        return s ^ (1 << m), sign

    def apply_cd(m, s):
        if (s >> m) & 1:
            return None, 0
        sign = (-1) ** bin(s & ((1 << m) - 1)).count("1")
        return s | (1 << m), sign

    for s in range(dim):
        n_up = [(s >> i) & 1 for i in range(L)]
        n_dn = [(s >> (L + i)) & 1 for i in range(L)]
        e = U * sum(n_up[i] * n_dn[i] for i in range(L))
        e += V * sum((n_up[i] + n_dn[i]) * (n_up[(i + 1) % L] + n_dn[(i + 1) % L]) for i in range(L))
        H[s, s] += e
        for spin in (0, L):
            for i in range(L):
                j = (i + 1) % L
                for a, b in ((i, j), (j, i)):  # c+_a c_b
                    s1, g1 = apply_c(spin + b, s)
                    if s1 is None:
                        continue
                    s2, g2 = apply_cd(spin + a, s1)
                    if s2 is None:
                        continue
                    H[s2, s] += -t * g1 * g2
    return H


@pytest.mark.parametrize("L,nu,nd", [(4, 2, 2), (4, 1, 2), (5, 2, 3)])
def test_hubbard_sector_matches_fock_space(L, nu, nd):
    t, U, V = 1.0, 4.0, 1.0
    Hs = hubbard_ring(L, nu, nd, t, U, V).to_dense()
    F = _fock_hamiltonian(L, t, U, V)
    up = sector_basis(L, nu)
    dn = sector_basis(L, nd)
    fock = (up[:, None] | (dn[None, :] << L)).ravel()
    assert np.array_equal(Hs, F[np.ix_(fock, fock)])
    assert np.allclose(Hs, Hs.T)


def test_hubbard_config3_counts():
    # the 14-site, 7+7 sector is checked for its closed-form size only (building it takes seconds)
    from math import comb

    assert comb(14, 7) ** 2 == 11778624
    H = hubbard_ring(8, 4, 4)
    assert H.n == comb(8, 4) ** 2
    assert _sorted_unique_rows(H)


@pytest.mark.slow
def test_hubbard_config3_full():
    p = config3_hubbard()
    assert p.H.n == 11778624 and p.H.nnz == 189364032
    assert abs(np.linalg.norm(p.B[0]) - 1) < 1e-12
