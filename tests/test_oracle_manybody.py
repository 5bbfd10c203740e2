"""Pins of the many-electron reference against facts outside it (CPU only).

* canonical anticommutation: {c_i, c+_j} = delta_ij and {c_i, c_j} = 0 on sector vectors
  (both spins, the ring's first and last sites);
* c+_i c_i is the occupation number of mode i;
* the hopping part of the sector matrix of workloads.hubbard (an independent construction)
  equals -t sum_i (c+_{i+1} c_i + c+_i c_{i+1}) composed from the operators;
* the free ring (U = V = 0) has the closed-form ground energy of filled periodic
  single-particle levels (which the Jordan-Wigner sign of the closing bond ensures);
* the projected resolvent equals its Lehmann sum over eigenpairs and its large-|z| expansion,
  and the removal weight of c_{0,up}|psi0> is the filling N_up / L.
"""

import numpy as np
import pytest

from oracle import manybody as MB
from workloads import hubbard_ring


def _rand(L, nu, nd, seed):
    D = len(MB.basis(L, nu)) * len(MB.basis(L, nd))
    return np.random.default_rng(seed).normal(size=D)


@pytest.mark.parametrize("spin", [0, 1])
def test_anticommutation(spin):
    L, nu, nd = 6, 3, 2
    x = _rand(L, nu, nd, 1)
    for i in (0, 2, L - 1):
        for j in (0, 3, L - 1):
            # c_i c+_j x + c+_j c_i x
            a, s1 = MB.fermion_op(L, nu, nd, j, spin, True, x)
            a, _ = MB.fermion_op(L, *s1, i, spin, False, a)
            b, s2 = MB.fermion_op(L, nu, nd, i, spin, False, x)
            b, _ = MB.fermion_op(L, *s2, j, spin, True, b)
            expect = x if i == j else np.zeros_like(x)
            assert np.max(np.abs(a + b - expect)) < 1e-14, (i, j)
            # c_i c_j x + c_j c_i x = 0
            a, s1 = MB.fermion_op(L, nu, nd, j, spin, False, x)
            a, _ = MB.fermion_op(L, *s1, i, spin, False, a)
            b, s2 = MB.fermion_op(L, nu, nd, i, spin, False, x)
            b, _ = MB.fermion_op(L, *s2, j, spin, False, b)
            assert np.max(np.abs(a + b)) < 1e-14
    # opposite spins anticommute too
    a, s1 = MB.fermion_op(L, nu, nd, 1, 1, False, x)
    a, _ = MB.fermion_op(L, *s1, 4, 0, False, a)
    b, s2 = MB.fermion_op(L, nu, nd, 4, 0, False, x)
    b, _ = MB.fermion_op(L, *s2, 1, 1, False, b)
    assert np.max(np.abs(a + b)) < 1e-14


def test_number_operator():
    L, nu, nd = 5, 2, 3
    x = _rand(L, nu, nd, 2)
    up, dn = MB.basis(L, nu), MB.basis(L, nd)
    for spin, pats in ((0, up), (1, dn)):
        for i in range(L):
            y, s = MB.fermion_op(L, nu, nd, i, spin, False, x)
            y, _ = MB.fermion_op(L, *s, i, spin, True, y)
            occ = (pats >> i) & 1
            n_i = np.repeat(occ, len(dn)) if spin == 0 else np.tile(occ, len(up))
            assert np.array_equal(y, n_i * x)


@pytest.mark.parametrize("L,nu,nd", [(6, 3, 3), (7, 2, 4)])
def test_hopping_from_operators_equals_sector_matrix(L, nu, nd):
    t = 1.0
    Hc = hubbard_ring(L, nu, nd, t=t, U=0.0, V=0.0)
    x = _rand(L, nu, nd, 3)
    y = np.zeros_like(x)
    for spin in (0, 1):
        for i in range(L):
            j = (i + 1) % L
            for a_, b_ in ((i, j), (j, i)):
                # c+_a c_b x
                w, s = MB.fermion_op(L, nu, nd, b_, spin, False, x)
                w, _ = MB.fermion_op(L, *s, a_, spin, True, w)
                y -= t * w
    ref = Hc.to_dense() @ x
    assert np.max(np.abs(y - ref)) < 1e-12


@pytest.mark.parametrize("L,nu,nd", [(6, 3, 2), (7, 2, 3)])
def test_free_ring_ground_state_closed_form(L, nu, nd):
    """U = V = 0: free fermions on a periodic ring, each species filling its lowest levels
    -2t cos(2 pi m / L).  In the occupation basis the bond that closes the ring carries
    (-1)^(N-1), which is what keeps the fermions periodic; without it an even count would see
    antiperiodic levels and a different energy."""
    t = 1.0
    Hc = hubbard_ring(L, nu, nd, t=t, U=0.0, V=0.0)
    E0, psi, _ = MB.ground_state(Hc.to_dense())

    def fill(n):
        eps = np.sort(-2 * t * np.cos(2 * np.pi * np.arange(L) / L))
        return eps[:n].sum()

    assert abs(E0 - (fill(nu) + fill(nd))) < 1e-12
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-14


def _golden(name):
    import os

    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v)
    return vals


def test_sector_dimension_of_the_papers_many_electron_problem():
    """The S_z = 0 sector size that Sec. 4.2 states for its many-electron problem, from the
    reference's basis enumeration (16 modes per spin, 6 electrons per spin)."""
    g = _golden("sector_dimension_sec4_2.txt")
    up = MB.basis(g["modes_per_spin"], g["electrons_per_spin"])
    assert len(up) ** 2 == g["dimension"]
    assert np.all(np.diff(up) > 0)  # increasing patterns, each with 6 bits set
    assert all(bin(int(s)).count("1") == g["electrons_per_spin"] for s in up[:: max(1, len(up) // 97)])


def test_projected_resolvent_spectral_form_and_removal_sum_rule():
    """<b|(z - H)^{-1}|b> equals the Lehmann sum over eigenpairs (v_a . b)^2 / (z - e_a); it
    decays as |b|^2 / z + b^T H b / z^2 at large |z|; and for b = c_{0,up}|psi0> of the
    translation-invariant ring the total removal weight |b|^2 is the up-spin filling N_up / L."""
    L, nu, nd = 6, 3, 3
    D = hubbard_ring(L, nu, nd, t=1.0, U=4.0, V=1.0).to_dense()
    E0, psi, E1 = MB.ground_state(D)
    assert E1 - E0 > 1e-6  # nondegenerate, so psi0 is translation invariant
    b, sec = MB.fermion_op(L, nu, nd, 0, 0, False, psi)
    assert sec == (nu - 1, nd)
    assert abs(b @ b - nu / L) < 1e-12
    Dm = hubbard_ring(L, *sec, t=1.0, U=4.0, V=1.0).to_dense()
    z = E0 - np.linspace(-6, 6, 13) + 0.2j
    G = MB.projected_resolvent(Dm, b, z)
    e, v = np.linalg.eigh(Dm)
    w = (v.T @ b) ** 2
    lehmann = np.array([np.sum(w / (zk - e)) for zk in z])
    assert np.max(np.abs(G - lehmann)) < 1e-11 * np.max(np.abs(G))
    zb = np.array([1e4 + 3e3j, -2e4 + 1e3j])
    Gb = MB.projected_resolvent(Dm, b, zb)
    asym = (b @ b) / zb + (b @ Dm @ b) / zb**2
    assert np.max(np.abs(Gb - asym) / np.abs(asym)) < 1e-6
