"""Pins of the Krylov-subspace (Lanczos) reference against facts outside it (CPU only).

* spectral moments: a Krylov subspace of dimension m reproduces <j|H^k|j> for k < 2m
  (a property of the orthonormal three-term basis, checked against repeated products);
* full dimension: with m = n the subspace Green's function is the exact (z - H)^{-1}_jj
  (dense inverse);
* a ring of sites with hopping -1 seen from one site has the closed-form coefficients
  a_n = 0, b = sqrt(2), 1, 1, ... while the walk has not wrapped around;
* an invariant subspace (|j> inside a 3-site block) stops the recurrence at m = 3, and
  the result is then exact.
"""

import numpy as np
import pytest

from oracle import krylov as K
from workloads import random_sparse_symmetric
from workloads.csr import coo_to_csr


def _ring(L, hop=-1.0):
    i = np.arange(L)
    rows = np.concatenate([i, (i + 1) % L])
    cols = np.concatenate([(i + 1) % L, i])
    return coo_to_csr(L, rows, cols, np.full(2 * L, hop))


@pytest.mark.parametrize("m", [1, 3, 8])
def test_moments_of_the_subspace_equal_those_of_h(m):
    rng = np.random.default_rng(5)
    H = random_sparse_symmetric(60, 0.1, rng, diag_scale=1.0)
    Hd = H.to_dense()
    Hd = Hd / np.abs(np.linalg.eigvalsh(Hd)).max()
    Hs = coo_to_csr(60, *np.nonzero(Hd), Hd[np.nonzero(Hd)])
    j = 7
    a, b = K.lanczos(Hs, j, m)
    assert len(a) == m
    T = K.reduced_hamiltonian(a, b)
    v = np.zeros(60)
    v[j] = 1.0
    hv = v.copy()
    Tk = np.eye(m)
    for k in range(2 * m):
        # <j|H^k|j> from repeated products, (T^k)_11 from the subspace
        assert abs(Tk[0, 0] - v @ hv) < 1e-12, k
        hv = Hd @ hv
        Tk = Tk @ T


def test_full_dimension_gives_the_exact_greens_function():
    rng = np.random.default_rng(6)
    n = 14
    H = random_sparse_symmetric(n, 0.5, rng, diag_scale=2.0)
    z = np.linspace(-4, 4, 9) + 0.1j
    for j in (0, 5, 13):
        a, b = K.lanczos(H, j, n)
        assert len(a) == n
        G = K.greens_from_subspace(a, b, z)
        exact = np.array([np.linalg.inv(zk * np.eye(n) - H.to_dense())[j, j] for zk in z])
        assert np.max(np.abs(G - exact) / np.abs(exact)) < 1e-10


def test_ring_has_closed_form_coefficients():
    a, b = K.lanczos(_ring(41), 0, 15)
    assert np.max(np.abs(a)) < 1e-15
    assert abs(b[0] - np.sqrt(2.0)) < 1e-15
    assert np.max(np.abs(b[1:] - 1.0)) < 1e-14


def test_invariant_subspace_stops_the_recurrence():
    # sites 0..2 form a chain decoupled from a random block on sites 3..19
    rng = np.random.default_rng(7)
    rest = random_sparse_symmetric(17, 0.4, rng, diag_scale=1.0)
    rows = [0, 1, 1, 2, 0, 1, 2] + list(np.repeat(np.arange(17), np.diff(rest.row_ptr)) + 3)
    cols = [1, 0, 2, 1, 0, 1, 2] + list(rest.col + 3)
    vals = [-1.0, -1.0, -0.5, -0.5, 0.3, -0.2, 0.1] + list(rest.val)
    H = coo_to_csr(20, np.array(rows), np.array(cols), np.array(vals))
    a, b = K.lanczos(H, 0, 10)
    assert len(a) == 3
    z = np.array([-1.0 + 0.05j, 0.2 + 0.3j, 2.0 + 0.01j])
    exact = np.array([np.linalg.inv(zk * np.eye(20) - H.to_dense())[0, 0] for zk in z])
    assert np.max(np.abs(K.greens_from_subspace(a, b, z) - exact) / np.abs(exact)) < 1e-12


def test_start_vector_subspace_reaches_the_exact_projected_resolvent():
    """From a real start vector b: at full dimension |b|^2 [(z - T)^{-1}]_11 is b^T (z - H)^{-1} b
    (the dense definition), and the moments b^T H^k b equal |b|^2 (T^k)_11 for k < 2m."""
    rng = np.random.default_rng(12)
    n = 18
    H = random_sparse_symmetric(n, 0.4, rng, diag_scale=2.0)
    D = H.to_dense()
    b = rng.normal(size=n)
    z = np.linspace(-4, 4, 9) + 0.3j
    G = K.krylov_greens_vec(H, z, b, n)
    exact = np.array([b @ np.linalg.solve(zk * np.eye(n) - D, b.astype(complex)) for zk in z])
    assert np.max(np.abs(G - exact) / np.abs(exact)) < 1e-9
    m = 5
    a, c = K.lanczos_from(H, b / np.linalg.norm(b), m)
    T = K.reduced_hamiltonian(a, c)
    nb2 = b @ b
    hv, tk = b.copy(), np.eye(len(a))[0]
    for k in range(2 * m):
        assert abs(b @ hv - nb2 * tk[0]) < 1e-9 * max(1.0, abs(b @ hv))
        hv = D @ hv
        tk = T @ tk
