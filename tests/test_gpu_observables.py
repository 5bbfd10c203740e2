"""Density matrix, band energy, backward and autograd through the HIP library,
against the FP64 oracle, dense references and finite differences."""

import numpy as np
import pytest

from oracle import oracle as O
from workloads import diamond, random_sparse_symmetric
from workloads.lattices import diamond_entry_map, diamond_geometry

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _S():
    import paper_0802_0748_amd as S

    return S


def _contour(H, nq):
    lo, _ = O.gershgorin(H)
    return lo - 1.0, 0.0, nq


def test_density_matrix_energy_matches_oracle():
    S = _S()
    Hc, _ = diamond(1, 1, 1, np.random.default_rng(4))
    e_lo, mu, nq = _contour(Hc, 48)
    z, w = S.contour(e_lo, mu, nq)
    H = S.Hamiltonian.from_csr(Hc)
    out = S.density_matrix_energy(H, z, w, want_rho=True, want_grad=True, tol=1e-13, max_iter=3000, rhs_batch=7)
    ref = O.density_matrix_energy(Hc, z, w, tol=1e-13, max_iter=3000)
    assert abs(out["E"].item() - ref["E"]) < 1e-10 * max(1, abs(ref["E"]))
    assert np.max(np.abs(out["rho"].cpu().numpy() - ref["rho"])) < 1e-10
    assert np.max(np.abs(out["grad"].cpu().numpy() - ref["grad"])) < 1e-9 * max(1, np.max(np.abs(ref["grad"])))


def test_backward_through_greens_diag_matches_formula():
    """dL/dH_ab = Re sum conj(g_kj) x_kj[a] x_kj[b], with x from the oracle and random g."""
    S = _S()
    rng = np.random.default_rng(1)
    Hc = random_sparse_symmetric(150, 0.04, rng, diag_scale=2.0)
    z = np.linspace(-2, 2, 5) + 0.2j
    idx = np.array([3, 77, 149])
    H = S.Hamiltonian.from_csr(Hc)
    G, rep, tape, rc = S.greens_diag(H, z, idx, tol=1e-13, max_iter=3000, keep_tape=True)
    g = rng.normal(size=(len(z), len(idx))) + 1j * rng.normal(size=(len(z), len(idx)))
    grad = S.backward(tape, torch.from_numpy(g).cuda()).cpu().numpy()
    rows = np.repeat(np.arange(Hc.n), np.diff(Hc.row_ptr))
    ref = np.zeros(Hc.nnz)
    for c, j in enumerate(idx):
        X = O.shifted_cocg(Hc, z, O.unit(Hc.n, j), tol=1e-13, max_iter=3000)["X"]
        assert np.max(np.abs(G.cpu().numpy()[:, c] - X[:, j])) < 1e-10
        for k in range(len(z)):
            ref += np.real(np.conj(g[k, c]) * X[k][rows] * X[k][Hc.col])
    assert np.max(np.abs(grad - ref)) < 1e-9 * max(1, np.max(np.abs(ref)))


def test_greens_diag_autograd_matches_dense_torch():
    """torch.autograd through GreensDiag against autograd through a dense complex inverse (CPU)."""
    S = _S()
    from paper_0802_0748_amd.autograd import greens_diag

    rng = np.random.default_rng(2)
    Hc = random_sparse_symmetric(60, 0.08, rng, diag_scale=2.0)
    z = np.linspace(-1.5, 1.5, 4) + 0.3j
    idx = np.array([0, 17, 59])
    H = S.Hamiltonian.from_csr(Hc)
    vals = torch.tensor(Hc.val, dtype=torch.float64, requires_grad=True)
    G = greens_diag(vals, H, z, idx, tol=1e-13, max_iter=3000)
    wgt = torch.from_numpy(rng.normal(size=G.shape) + 1j * rng.normal(size=G.shape)).cuda()
    loss = (torch.abs(G) ** 2).sum() + torch.real(wgt * G).sum()
    loss.backward()
    # dense reference on the CPU
    rows = torch.from_numpy(np.repeat(np.arange(Hc.n), np.diff(Hc.row_ptr)))
    cols = torch.from_numpy(Hc.col)
    v2 = torch.tensor(Hc.val, dtype=torch.float64, requires_grad=True)
    A = torch.zeros((Hc.n, Hc.n), dtype=torch.float64).index_put((rows, cols), v2)
    Gs = []
    for zk in z:
        Ginv = torch.linalg.inv(zk * torch.eye(Hc.n, dtype=torch.complex128) - A.to(torch.complex128))
        Gs.append(Ginv[idx, idx])
    Gd = torch.stack(Gs)
    assert torch.max(torch.abs(Gd - G.detach().cpu())) < 1e-10
    loss_d = (torch.abs(Gd) ** 2).sum() + torch.real(wgt.cpu() * Gd).sum()
    loss_d.backward()
    assert torch.max(torch.abs(vals.grad - v2.grad)) < 1e-8 * max(1.0, torch.max(torch.abs(v2.grad)).item())


def _diamond_model(cells, seed):
    Hc, geo = diamond(*cells, np.random.default_rng(seed))
    kind, bond, o1, o2 = diamond_entry_map(Hc, geo["bonds"])
    _, bonds, vec0 = diamond_geometry(*cells)
    t = lambda a: torch.from_numpy(np.asarray(a))
    model = dict(vec0=t(vec0), bonds=t(bonds), blocks=t(geo["blocks"]), kind=t(kind), bond=t(bond), o1=t(o1),
                 o2=t(o2), onsite=t(Hc.val.copy()))
    return Hc, geo, model


def _values(model, disp):
    from paper_0802_0748_amd.autograd import hopping_values

    m = model
    return hopping_values(m["vec0"], disp, m["bonds"], m["blocks"], m["kind"], m["bond"], m["o1"], m["o2"],
                          m["onsite"])


def test_band_energy_forces_match_finite_differences():
    """Forces -dE/dR through t(r) = exp(-2 (r - r0)) on the 32-atom cell, against central
    differences (h = 1e-5) of the GPU band energy with the contour held fixed (5 coordinates), and
    of the dense CPU evaluation of the same quadrature energy (all 96 coordinates)."""
    S = _S()
    from paper_0802_0748_amd.autograd import band_energy

    Hc, geo, model = _diamond_model((2, 2, 1), 0)
    e_lo, mu, nq = _contour(Hc, 128)
    z, w = S.contour(e_lo - 2.0, mu, nq)
    H = S.Hamiltonian.from_csr(Hc)
    disp0 = torch.from_numpy(geo["displacement"].copy())
    disp = disp0.clone().requires_grad_(True)
    E = band_energy(_values(model, disp), H, z, w, tol=1e-13, max_iter=5000)
    E.backward()
    forces = -disp.grad.numpy()
    h = 1e-5
    rng = np.random.default_rng(0)
    for a, c in [(0, 0), (5, 1), (17, 2), (31, 0), (int(rng.integers(32)), int(rng.integers(3)))]:
        Es = []
        for sgn in (+1, -1):
            d = disp0.clone()
            d[a, c] += sgn * h
            Es.append(band_energy(_values(model, d), H, z, w, tol=1e-13, max_iter=5000).item())
        fd = -(Es[0] - Es[1]) / (2 * h)
        assert abs(fd - forces[a, c]) < 1e-6 * max(1.0, abs(forces[a, c])), (a, c, fd, forces[a, c])
    # all 96 coordinates: central differences of the same quadrature energy evaluated densely on
    # the CPU, E = Re sum_k w_k z_k sum_i 1/(z_k - lambda_i) over the eigenvalues of H(R)
    rows = np.repeat(np.arange(Hc.n), np.diff(Hc.row_ptr))
    zz, ww = np.asarray(z), np.asarray(w)

    def e_dense(d):
        A = np.zeros((Hc.n, Hc.n))
        A[rows, Hc.col] = _values(model, d).numpy()
        lam = np.linalg.eigvalsh(A)
        return float(np.real(np.sum(ww * zz * np.sum(1.0 / (zz[:, None] - lam[None, :]), axis=1))))

    assert abs(e_dense(disp0) - E.item()) < 1e-10 * max(1.0, abs(E.item()))
    fd_all = np.zeros_like(forces)
    for a in range(forces.shape[0]):
        for c in range(3):
            dp, dm = disp0.clone(), disp0.clone()
            dp[a, c] += h
            dm[a, c] -= h
            fd_all[a, c] = -(e_dense(dp) - e_dense(dm)) / (2 * h)
    assert forces.shape == (32, 3)
    assert np.max(np.abs(fd_all - forces)) < 1e-6 * max(1.0, np.max(np.abs(forces))), np.max(np.abs(fd_all - forces))


def test_band_energy_gradient_matches_dense_autograd():
    """dE/dR on the 64-atom cell against FP64 torch autograd through dense complex inverses."""
    S = _S()
    from paper_0802_0748_amd.autograd import band_energy

    Hc, geo, model = _diamond_model((2, 2, 2), 3)
    e_lo, mu, nq = _contour(Hc, 64)
    z, w = S.contour(e_lo - 2.0, mu, nq)
    H = S.Hamiltonian.from_csr(Hc)
    disp = torch.from_numpy(geo["displacement"].copy()).requires_grad_(True)
    E = band_energy(_values(model, disp), H, z, w, tol=1e-13, max_iter=5000)
    E.backward()
    g_gpu = disp.grad.clone()
    d2 = torch.from_numpy(geo["displacement"].copy()).requires_grad_(True)
    vals = _values(model, d2)
    rows = torch.from_numpy(np.repeat(np.arange(Hc.n), np.diff(Hc.row_ptr)))
    A = torch.zeros((Hc.n, Hc.n), dtype=torch.float64).index_put((rows, torch.from_numpy(Hc.col)), vals)
    Ac = A.to(torch.complex128)
    I = torch.eye(Hc.n, dtype=torch.complex128)
    Ed = 0.0
    for zk, wk in zip(z, w):
        G = torch.linalg.inv(zk * I - Ac)
        Ed = Ed + torch.real(wk * zk * torch.diagonal(G).sum())
    assert abs(Ed.item() - E.item()) < 1e-9 * max(1.0, abs(Ed.item()))
    Ed.backward()
    assert torch.max(torch.abs(g_gpu - d2.grad)) < 1e-8 * max(1.0, torch.max(torch.abs(d2.grad)).item())


def test_backward_after_the_matrix_is_freed():
    """A tape keeps the matrix it was recorded on: freeing the caller's handle (csr_free through
    the C ABI) before backward() still gives the gradient of the live matrix, bit for bit; a
    temporary Hamiltonian passed to the autograd wrapper works the same way."""
    S = _S()
    from paper_0802_0748_amd.autograd import greens_diag

    rng = np.random.default_rng(12)
    Hc = random_sparse_symmetric(120, 0.05, rng, diag_scale=2.0)
    z = np.linspace(-2, 2, 4) + 0.3j
    idx = np.array([1, 50, 119])
    g = torch.from_numpy(rng.normal(size=(len(z), len(idx))) + 1j * rng.normal(size=(len(z), len(idx)))).cuda()
    H_keep = S.Hamiltonian.from_csr(Hc)
    _, _, tape_keep, _ = S.greens_diag(H_keep, z, idx, tol=1e-13, max_iter=3000, keep_tape=True)
    ref = S.backward(tape_keep, g).cpu().numpy()
    H_tmp = S.Hamiltonian.from_csr(Hc)
    _, _, tape, _ = S.greens_diag(H_tmp, z, idx, tol=1e-13, max_iter=3000, keep_tape=True)
    H_tmp.close()  # csr_free: the tape still holds the matrix
    tape.hamiltonian = None
    del H_tmp
    got = S.backward(tape, g).cpu().numpy()
    tape.close()
    assert np.array_equal(got, ref)
    # the autograd path with a temporary Hamiltonian
    vals = torch.tensor(Hc.val, dtype=torch.float64, requires_grad=True)
    G = greens_diag(vals, S.Hamiltonian.from_csr(Hc), z, idx, tol=1e-13, max_iter=3000)
    torch.real(torch.sum(torch.conj(g) * G)).backward()
    vals2 = torch.tensor(Hc.val, dtype=torch.float64, requires_grad=True)
    G2 = greens_diag(vals2, H_keep, z, idx, tol=1e-13, max_iter=3000)
    torch.real(torch.sum(torch.conj(g) * G2)).backward()
    assert torch.equal(vals.grad, vals2.grad)


def test_autograd_refuses_unconverged_pairs():
    """Observables built on pairs that stopped unconverged are refused by the autograd wrappers
    (ENOCONV), unless the caller allows them; the per-pair report says which pairs."""
    S = _S()
    from paper_0802_0748_amd._capi import ENOCONV, ScocgError
    from paper_0802_0748_amd.autograd import band_energy, greens_diag

    rng = np.random.default_rng(13)
    Hc = random_sparse_symmetric(80, 0.08, rng, diag_scale=2.0)
    H = S.Hamiltonian.from_csr(Hc)
    z = np.linspace(-2, 2, 4) + 0.05j
    vals = torch.tensor(Hc.val, dtype=torch.float64, requires_grad=True)
    with pytest.raises(ScocgError) as ei:
        greens_diag(vals, H, z, [0, 3], tol=1e-12, max_iter=5)
    assert ei.value.code == ENOCONV
    report = {}
    G = greens_diag(vals, H, z, [0, 3], tol=1e-12, max_iter=5, allow_noconv=True, report=report)
    assert report["rc"] == ENOCONV and np.all(report["status"] == ENOCONV)
    assert G.shape == (4, 2)
    e_lo, mu, nq = _contour(Hc, 16)
    zq, wq = S.contour(e_lo, mu, nq)
    with pytest.raises(ScocgError):
        band_energy(vals, H, zq, wq, tol=1e-12, max_iter=3)


def test_density_matrix_energy_refuses_duplicate_columns():
    """A column listed twice would be accumulated twice into rho (and raced on within a batch):
    refused with EINVAL before any work."""
    S = _S()
    from paper_0802_0748_amd._capi import ScocgError

    rng = np.random.default_rng(14)
    Hc = random_sparse_symmetric(40, 0.1, rng, diag_scale=2.0)
    H = S.Hamiltonian.from_csr(Hc)
    e_lo, mu, nq = _contour(Hc, 8)
    zq, wq = S.contour(e_lo, mu, nq)
    with pytest.raises(ScocgError, match="more than once"):
        S.density_matrix_energy(H, zq, wq, rhs_idx=[3, 7, 3], tol=1e-10, max_iter=2000)


def test_gradient_and_backward_with_rows_wider_than_32():
    """Rows of 40-60 stored entries (segments of 32 per row in the pair contraction): rho, E and
    dE/dH against the oracle, and backward through G against the formula with oracle solutions."""
    S = _S()
    rng = np.random.default_rng(15)
    Hc = random_sparse_symmetric(110, 0.45, rng, diag_scale=3.0)
    widths = np.diff(Hc.row_ptr)
    assert widths.max() > 40 and widths.min() > 32
    H = S.Hamiltonian.from_csr(Hc)
    e_lo, mu, nq = _contour(Hc, 24)
    zq, wq = S.contour(e_lo, mu, nq)
    cols = np.array([0, 5, 33, 60, 109])
    out = S.density_matrix_energy(H, zq, wq, rhs_idx=cols, want_rho=True, want_grad=True, tol=1e-13, max_iter=4000,
                                  rhs_batch=2)
    ref = O.density_matrix_energy(Hc, zq, wq, rhs_idx=cols, tol=1e-13, max_iter=4000)
    assert abs(out["E"].item() - ref["E"]) < 1e-10 * max(1, abs(ref["E"]))
    assert np.max(np.abs(out["rho"].cpu().numpy() - ref["rho"])) < 1e-10
    assert np.max(np.abs(out["grad"].cpu().numpy() - ref["grad"])) < 1e-9 * max(1, np.max(np.abs(ref["grad"])))
    z = np.linspace(-3, 3, 3) + 0.4j
    G, _, tape, _ = S.greens_diag(H, z, cols[:3], tol=1e-13, max_iter=4000, keep_tape=True)
    g = rng.normal(size=(len(z), 3)) + 1j * rng.normal(size=(len(z), 3))
    grad = S.backward(tape, torch.from_numpy(g).cuda()).cpu().numpy()
    rows = np.repeat(np.arange(Hc.n), widths)
    expect = np.zeros(Hc.nnz)
    for c, j in enumerate(cols[:3]):
        X = O.shifted_cocg(Hc, z, O.unit(Hc.n, int(j)), tol=1e-13, max_iter=4000)["X"]
        for k in range(len(z)):
            expect += np.real(np.conj(g[k, c]) * X[k][rows] * X[k][Hc.col])
    assert np.max(np.abs(grad - expect)) < 1e-9 * max(1, np.max(np.abs(expect)))


def test_band_energy_gradient_full_size_columns_match_oracle():
    """The band-energy workload at full size: the 8x8x8 diamond cell (16384 orbitals), the
    128-node contour with the Fermi level at 0 (its end node 0.004 above the real axis, where
    the spectrum is dense), production tolerance 1e-8.  For eight columns spread over the matrix,
    rho on their stored entries, their band-energy part and their contribution to dE/dH (on
    every stored entry) agree with the oracle (eight columns solved in parallel threads) within
    the error bound both answers' residuals give (Sec. 3.4: |x - x*| <= ||r|| / Im z per pair;
    the GPU's true residuals are at most 20 tol, as the full-size diamond checks show)."""
    import time
    from concurrent.futures import ThreadPoolExecutor

    from workloads import config2_diamond

    S = _S()
    p = config2_diamond()
    Hc = p.H
    lo, _ = O.gershgorin(Hc)
    zq, wq = S.contour(lo - 1.0, 0.0, 128)
    cols = np.array([0, 1, 2, 3, 5000, 8191, 12000, 16383])
    tol = 1e-8
    H = S.Hamiltonian.from_csr(Hc)
    t0 = time.perf_counter()
    out = S.density_matrix_energy(H, zq, wq, rhs_idx=cols, want_rho=True, want_grad=True, tol=tol, max_iter=60000,
                                  allow_noconv=False)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=8) as ex:
        parts = list(ex.map(lambda c: O.density_matrix_energy(Hc, zq, wq, rhs_idx=[c], want_residuals=True, tol=tol,
                                                              max_iter=60000), cols))
    t_orc = time.perf_counter() - t0
    E_orc = sum(q["E"] for q in parts)
    rho_orc = sum(q["rho"] for q in parts)
    grad_orc = sum(q["grad"] for q in parts)
    r_orc = np.array([q["res_true"][0] for q in parts])  # [8, 128]
    d = (20 * tol + r_orc) / zq.imag[None, :]  # per-pair bound on |x_gpu - x_orc|
    rows = np.repeat(np.arange(Hc.n), np.diff(Hc.row_ptr))
    rho_gpu = out["rho"].cpu().numpy()
    grad_gpu = out["grad"].cpu().numpy()
    dE = abs(out["E"].item() - E_orc)
    E_bound = float(np.sum(np.abs(wq * zq)[None, :] * d))
    drho = np.abs(rho_gpu - rho_orc)
    rho_bound = np.zeros(Hc.nnz)
    for c, j in enumerate(cols):
        rho_bound[Hc.col == j] = np.sum(np.abs(wq) * d[c])
    dgrad = np.abs(grad_gpu - grad_orc)
    grad_bound = float(np.sum(np.abs(wq * zq)[None, :] * d * (2.0 / zq.imag[None, :] + d)))
    print(f"8 columns: GPU {t_gpu:.1f} s, oracle {t_orc:.1f} s; |dE| {dE:.1e} (bound {E_bound:.1e}), max |drho| "
          f"{drho.max():.1e}, max |dgrad| {dgrad.max():.1e} (bound {grad_bound:.1e}), max oracle residual "
          f"{r_orc.max():.1e}", flush=True)
    assert np.all(r_orc < 20 * tol)
    assert dE <= E_bound
    assert np.all(drho <= rho_bound * (1 + 1e-9) + 1e-15)
    assert np.all(rho_gpu[~np.isin(Hc.col, cols)] == 0)
    assert dgrad.max() <= grad_bound
