"""Ground state and single-particle excitations of the Hubbard ring on the GPU
(ground_state, hubbard_fermion_op) against the many-electron reference."""

import numpy as np
import pytest

from oracle import manybody as MB
from workloads import hubbard_ring

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _S():
    import paper_0802_0748_amd as S

    return S


def _crand(D, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=D) + 1j * rng.normal(size=D)


@pytest.mark.parametrize("L,nu,nd", [(6, 3, 3), (7, 2, 4), (9, 4, 1)])
def test_fermion_operator_matches_reference_bitwise(L, nu, nd):
    S = _S()
    D = len(MB.basis(L, nu)) * len(MB.basis(L, nd))
    x = _crand(D, L)
    xt = torch.from_numpy(x).cuda()
    for site in (0, L // 2, L - 1):
        for spin in (0, 1):
            for create in (False, True):
                cnt = (nu if spin == 0 else nd) + (1 if create else -1)
                if not 0 <= cnt <= L:
                    continue
                y, sec = S.hubbard_fermion_op(L, nu, nd, site, spin, create, xt)
                ref, rsec = MB.fermion_op(L, nu, nd, site, spin, create, x)
                assert sec == rsec
                assert np.array_equal(y.cpu().numpy(), ref), (site, spin, create)


def test_hopping_composed_on_gpu_equals_sector_matrix():
    S = _S()
    L, nu, nd, t = 8, 4, 3, 1.0
    Hc = hubbard_ring(L, nu, nd, t=t, U=0.0, V=0.0)
    x = _crand(Hc.n, 4)
    xt = torch.from_numpy(x).cuda()
    y = torch.zeros_like(xt)
    for spin in (0, 1):
        for i in range(L):
            j = (i + 1) % L
            for a, b in ((i, j), (j, i)):
                w, sec = S.hubbard_fermion_op(L, nu, nd, b, spin, False, xt)
                w, _ = S.hubbard_fermion_op(L, *sec, a, spin, True, w)
                y -= t * w
    ref = Hc.to_dense() @ x
    assert np.max(np.abs(y.cpu().numpy() - ref)) < 1e-12


@pytest.mark.parametrize("L,nu,nd,U,V,steps", [(8, 4, 4, 4.0, 1.0, 120), (8, 4, 4, 4.0, 1.0, 16),
                                                (9, 4, 3, 2.0, 0.5, 120), (9, 4, 3, 2.0, 0.5, 16)])
def test_ground_state_matches_dense_diagonalization(L, nu, nd, U, V, steps):
    """With a short recurrence the Ritz vector is rough and inverse iteration does the work.
    A degenerate ground state (the 9-site sector's) is compared through its eigenspace."""
    S = _S()
    Hc = hubbard_ring(L, nu, nd, t=1.0, U=U, V=V)
    H = S.Hamiltonian.from_csr(Hc)
    x0 = np.random.default_rng(L).normal(size=Hc.n)
    psi, E0, E1, res, sweeps = S.ground_state(H, x0, nu=steps, tol=1e-10)
    e, vecs = np.linalg.eigh(Hc.to_dense())
    print(f"sector {L},{nu},{nd}, {steps} steps: E0 {E0:.12f} (dense {e[0]:.12f}), residual {res:.1e}, "
          f"sweeps {sweeps}")
    assert res <= 1e-10
    assert abs(E0 - e[0]) <= 1e-10 * max(1.0, abs(e[0]))
    p = psi.cpu().numpy()
    assert np.max(np.abs(p.imag)) == 0.0
    ground = vecs[:, np.abs(e - e[0]) < 1e-8]
    assert abs(np.linalg.norm(ground.T @ p.real) - 1.0) < 1e-9
    assert E1 >= E0 - 1e-9
    if steps < 20:
        assert sweeps >= 1


@pytest.mark.parametrize("steps", [120, 16])
def test_ground_state_matrix_free_equals_stored(steps):
    """The ground state on the matrix-free operator: its rows give the stored matrix's sums
    and the inverse-iteration solves its products, so psi and E are the same bits."""
    S = _S()
    L, nu, nd = 10, 5, 4
    Hc = hubbard_ring(L, nu, nd, t=1.0, U=4.0, V=1.0)
    Hm = S.Hamiltonian.from_csr(Hc)
    Ho = S.Hamiltonian.hubbard(L, nu, nd, t=1.0, U=4.0, V=1.0)
    x0 = np.random.default_rng(5).normal(size=Hc.n)
    pm, Em, E1m, rm, sm = S.ground_state(Hm, x0, nu=steps, tol=1e-10)
    po, Eo, E1o, ro, so = S.ground_state(Ho, x0, nu=steps, tol=1e-10)
    print(f"{steps} steps: E0 {Eo:.12f}, residual {ro:.1e}, sweeps {so}")
    assert (Eo, E1o, ro, so) == (Em, E1m, rm, sm)
    assert np.array_equal(po.cpu().numpy(), pm.cpu().numpy())
    assert ro <= 1e-10


def test_ionization_spectrum_from_the_ground_state():
    """b = c_{0,up}|psi0> in the sector with one up electron less; the ionization Green's
    function <b|((E0 - w) + i eta - H)^{-1}|b> over a range of energies, by the shifted COCG
    solver on b, against dense solves of the reference."""
    S = _S()
    L, nu, nd = 8, 4, 4
    Hc = hubbard_ring(L, nu, nd, t=1.0, U=4.0, V=1.0)
    H = S.Hamiltonian.from_csr(Hc)
    psi, E0, _, res, _ = S.ground_state(H, np.random.default_rng(1).normal(size=Hc.n), nu=120, tol=1e-11)
    b, sec = S.hubbard_fermion_op(L, nu, nd, 0, 0, False, psi)
    Hm = hubbard_ring(L, *sec, t=1.0, U=4.0, V=1.0)
    Hm_gpu = S.Hamiltonian.from_csr(Hm)
    w = np.linspace(-8, 8, 33)
    z = (E0 - w) + 0.1j
    X, rep, _, rc = S.shifted_cocg_solve(Hm_gpu, z, b[None, :], tol=1e-12, max_iter=20000)
    assert rc == 0
    G = (X[0] @ b).cpu().numpy()  # bilinear <b|x_k> (b is real)
    E_ref, psi_ref, _ = MB.ground_state(Hc.to_dense())
    sgn = np.sign(psi.cpu().numpy().real @ psi_ref)
    b_ref, _ = MB.fermion_op(L, nu, nd, 0, 0, False, sgn * psi_ref.astype(complex))
    ref = MB.projected_resolvent(Hm.to_dense(), b_ref.real, z)
    assert np.max(np.abs(G - ref) / np.abs(ref)) < 1e-8
    # the spectral weight sums to the occupation <psi0|n_{0,up}|psi0> = N_up / L on the ring
    assert abs(float((b.conj() @ b).real) - nu / L) < 1e-10


def test_affinity_spectrum_and_the_total_sum_rule():
    """b' = c+_{0,up}|psi0> in the sector with one up electron more: the addition Green's
    function <b'|((E0 + w) + i eta - H)^{-1}|b'> against dense solves of the reference; the
    removal and addition weights <b|b> + <b'|b'> add up to 1 (the anticommutator
    {c, c+} = 1 in the ground state), and both spectral functions are non-negative."""
    S = _S()
    L, nu, nd = 8, 4, 4
    Hc = hubbard_ring(L, nu, nd, t=1.0, U=4.0, V=1.0)
    H = S.Hamiltonian.hubbard(L, nu, nd, t=1.0, U=4.0, V=1.0)
    psi, E0, _, res, _ = S.ground_state(H, np.random.default_rng(2).normal(size=Hc.n), nu=120, tol=1e-11)
    b, sec_m = S.hubbard_fermion_op(L, nu, nd, 0, 0, False, psi)
    bp, sec_p = S.hubbard_fermion_op(L, nu, nd, 0, 0, True, psi)
    assert sec_p == (nu + 1, nd)
    w = np.linspace(-8, 8, 33)
    eta = 0.1
    Hp = S.Hamiltonian.hubbard(L, *sec_p, t=1.0, U=4.0, V=1.0)
    Xp, _, _, rc = S.shifted_cocg_solve(Hp, (E0 + w) + 1j * eta, bp[None, :], tol=1e-12, max_iter=20000)
    assert rc == 0
    Gp = (Xp[0] @ bp).cpu().numpy()
    E_ref, psi_ref, _ = MB.ground_state(Hc.to_dense())
    sgn = np.sign(psi.cpu().numpy().real @ psi_ref)
    bp_ref, _ = MB.fermion_op(L, nu, nd, 0, 0, True, sgn * psi_ref.astype(complex))
    Hp_dense = hubbard_ring(L, *sec_p, t=1.0, U=4.0, V=1.0).to_dense()
    ref = MB.projected_resolvent(Hp_dense, bp_ref.real, (E_ref + w) + 1j * eta)
    assert np.max(np.abs(Gp - ref) / np.abs(ref)) < 1e-8
    Xm, _, _, rc = S.shifted_cocg_solve(S.Hamiltonian.hubbard(L, *sec_m, t=1.0, U=4.0, V=1.0),
                                        (E0 - w) + 1j * eta, b[None, :], tol=1e-12, max_iter=20000)
    assert rc == 0
    Gm = (Xm[0] @ b).cpu().numpy()
    wm, wp = float((b.conj() @ b).real), float((bp.conj() @ bp).real)
    assert abs(wm + wp - 1.0) < 1e-12
    assert abs(wp - (1 - nu / L)) < 1e-10
    assert np.all(-Gm.imag >= 0) and np.all(-Gp.imag >= 0)


def test_ground_state_limits_and_bad_arguments():
    """No sweep allowed and a tolerance the short estimate cannot meet: ENOCONV, with the
    estimate still returned when asked for; invalid arguments of both calls are rejected."""
    from paper_0802_0748_amd._capi import ScocgError

    S = _S()
    L, nu, nd = 8, 4, 4
    H = S.Hamiltonian.hubbard(L, nu, nd, t=1.0, U=4.0, V=1.0)
    x0 = np.random.default_rng(3).normal(size=H.n)
    with pytest.raises(ScocgError):
        S.ground_state(H, x0, nu=6, tol=1e-12, max_sweeps=0)
    psi, E0, E1, res, sweeps = S.ground_state(H, x0, nu=6, tol=1e-12, max_sweeps=0, allow_noconv=True)
    assert sweeps == 0 and res > 1e-12 and np.isfinite(E0)
    assert abs(float((psi.conj() @ psi).real) - 1.0) < 1e-12
    for bad in [dict(nu=1), dict(nu=(1 << 20) + 1), dict(tol=0.0), dict(max_sweeps=-1)]:
        with pytest.raises(ScocgError):
            S.ground_state(H, x0, **bad)
    x = torch.from_numpy(_crand(H.n, 1)).cuda()
    for site, spin in [(-1, 0), (L, 0), (0, 2)]:
        with pytest.raises(ScocgError):
            S.hubbard_fermion_op(L, nu, nd, site, spin, False, x)
    with pytest.raises(ValueError):  # no sector with nine up electrons on eight sites
        S.hubbard_fermion_op(L, L, nd, 0, 0, True, torch.zeros(70, dtype=torch.complex128, device="cuda"))


def test_projected_greens_functions_carried_by_scalars():
    """greens_proj: <w|(z - H)^{-1}|b> with every shift carried by scalars (Sec. 3.3) for the
    removal part of the ground state, diagonal (w = b) and off-diagonal (w = c_{1,up}|psi0>),
    against dense solves of the reference; all shifts stored or a window of four; and in
    fixed-iteration mode against the full solutions' projections."""
    S = _S()
    L, nu, nd = 8, 4, 4
    Hc = hubbard_ring(L, nu, nd, t=1.0, U=4.0, V=1.0)
    H = S.Hamiltonian.hubbard(L, nu, nd, t=1.0, U=4.0, V=1.0)
    psi, E0, _, _, _ = S.ground_state(H, np.random.default_rng(4).normal(size=Hc.n), nu=120, tol=1e-11)
    b0, sec = S.hubbard_fermion_op(L, nu, nd, 0, 0, False, psi)
    b1, _ = S.hubbard_fermion_op(L, nu, nd, 1, 0, False, psi)
    Hm_dense = hubbard_ring(L, *sec, t=1.0, U=4.0, V=1.0).to_dense()
    Hm = S.Hamiltonian.hubbard(L, *sec, t=1.0, U=4.0, V=1.0)
    w = np.linspace(-8, 8, 33)
    z = (E0 - w) + 0.1j
    B = torch.stack([b0, b0])
    Wt = torch.stack([b0, b1])
    bn, b1n = b0.cpu().numpy(), b1.cpu().numpy()
    ref = []
    for zk in z:
        xk = np.linalg.solve(zk * np.eye(len(bn)) - Hm_dense, bn)
        ref.append([bn @ xk, b1n @ xk])
    ref = np.array(ref)
    for window in (0, 4):
        G, rep, _, rc = S.greens_proj(Hm, z, B, Wt, tol=1e-12, max_iter=20000, window=window)
        G = G.cpu().numpy()
        ok = rep["status"].T == 0  # [shift][rhs]
        print(f"window {window}: rc {rc}, converged {ok.sum()} of {ok.size}, switches {S.last_timing()['switches']}")
        if window == 0:
            assert rc == 0 and ok.all()
        assert ok.sum() >= ok.size // 2
        err = np.abs(G - ref) / np.abs(ref).max(axis=0)
        assert np.max(err[ok]) < 1e-8, (window, np.max(err[ok]))
    X, _, _, _ = S.shifted_cocg_solve(Hm, z, B[:1], fixed_iter=40, seed_index=3)
    Gf, _, _, _ = S.greens_proj(Hm, z, B[:1], Wt[:1], fixed_iter=40, seed_index=3)
    proj = (X[0] @ b0).cpu().numpy()
    assert np.max(np.abs(Gf.cpu().numpy()[:, 0] - proj) / np.abs(proj)) < 1e-10
