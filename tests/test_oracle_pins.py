"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: each check uses a textbook
routine (dense Gaussian elimination / eigendecomposition), a closed form, an
identity that holds in exact arithmetic, or a brute-force construction.
"""

import numpy as np
import pytest

from oracle import oracle as O
from workloads import config1_cubic, random_sparse_symmetric, simple_cubic


def _dense_solve(H, z, b):
    A = H.to_dense()
    return np.linalg.solve(z * np.eye(H.n) - A, b)


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(7)
    H = random_sparse_symmetric(36, 0.12, rng, diag_scale=1.5)
    z = np.linspace(-3.0, 3.0, 9) + 1j * np.array([0.05, 0.2, 0.1, 0.3, 0.05, 0.5, 0.1, 0.2, 0.08])
    return H, z


def test_converged_solution_equals_dense_solve(small):
    """Sec. 3.1 eq. lin_eq: x = (z - H)^{-1} b; dense Gaussian elimination is the definition."""
    H, z = small
    rng = np.random.default_rng(3)
    b = rng.normal(size=H.n) + 1j * rng.normal(size=H.n)
    out = O.shifted_cocg(H, z, b, tol=1e-13, max_iter=2000)
    assert out["ret"] == O.OK
    for k in range(len(z)):
        xd = _dense_solve(H, z[k], b)
        assert np.linalg.norm(out["X"][k] - xd) <= 1e-10 * np.linalg.norm(xd)


def test_fixed_iteration_matches_independent_cocg(small):
    """Shift invariance of the Krylov space (Sec. 3.1 eq. inv_KS) and collinear residuals
    (Sec. 3.3): after n steps the shifted iterate equals plain COCG on that shift."""
    H, z = small
    b = O.unit(H.n, 5) + 0.3 * O.unit(H.n, 11)
    n_it = 12
    out = O.shifted_cocg(H, z, b, fixed_iter=n_it, seed_index=2)
    for k in range(len(z)):
        ref = O.cocg(H, z[k], b, fixed_iter=n_it)
        assert ref["iters"] == n_it
        assert np.linalg.norm(out["X"][k] - ref["x"]) <= 1e-11 * np.linalg.norm(ref["x"])


def test_collinear_residual(small):
    """Sec. 3.3: the shifted residual b - (z_k - H) x_k equals the seed residual divided by pi_k."""
    H, z = small
    b = O.unit(H.n, 0)
    A = H.to_dense()
    for n_it in (1, 4, 9):
        out = O.shifted_cocg(H, z, b, fixed_iter=n_it, seed_index=4)
        for k in range(len(z)):
            rk = b - (z[k] * np.eye(H.n) - A) @ out["X"][k]
            assert np.linalg.norm(rk - out["r"] / out["pi"][k]) <= 1e-11 * np.linalg.norm(rk)


def test_seed_choice_and_switch_point_do_not_change_iterates(small):
    """Sec. 3.3 (seed switching keeps the computed information): the n-th iterate of every
    shift is independent of the seed and of where the seed is switched."""
    H, z = small
    b = O.unit(H.n, 2)
    n_it = 15
    ref = O.shifted_cocg(H, z, b, fixed_iter=n_it, seed_index=0)["X"]
    for seed, sw in ((3, None), (8, None), (0, (4, 6)), (5, (9, 1)), (1, (0, 7))):
        X = O.shifted_cocg(H, z, b, fixed_iter=n_it, seed_index=seed, force_switch=sw)["X"]
        for k in range(len(z)):
            assert np.linalg.norm(X[k] - ref[k]) <= 1e-11 * np.linalg.norm(ref[k])


def test_automatic_seed_switching_reaches_dense_solution():
    """Seed switching in production mode: the seed converges first (large eta), the
    others continue from a new seed and still reach the dense solution."""
    rng = np.random.default_rng(11)
    H = random_sparse_symmetric(48, 0.1, rng, diag_scale=2.0)
    z = np.array([0.0 + 1.0j, -1.0 + 0.02j, 0.5 + 0.05j, 1.5 + 0.01j, -0.3 + 0.2j])
    b = O.unit(H.n, 7)
    out = O.shifted_cocg(H, z, b, tol=1e-12, max_iter=2000, seed_index=0)
    assert out["ret"] == O.OK
    assert len(out["switches"]) >= 1
    for k in range(len(z)):
        xd = _dense_solve(H, z[k], b)
        assert np.linalg.norm(out["X"][k] - xd) <= 1e-9 * np.linalg.norm(xd)
    # the switch target is the active shift with the largest recursive residual; all
    # recorded iterations are increasing
    its = [s[0] for s in out["switches"]]
    assert its == sorted(its)


def test_default_seed_rule(small):
    H, z = small
    # smallest Im z: indices 0 and 4 (0.05); tie broken by distance of Re z to Tr(H)/n
    centre = np.trace(H.to_dense()) / H.n
    cand = [0, 4]
    expect = min(cand, key=lambda k: (abs(z[k].real - centre), k))
    assert O.default_seed(H, z) == expect


def test_error_bound_from_residual(small):
    """Sec. 3.4: the residual norm bounds the error of G.  For real-symmetric H,
    ||(z - H)^{-1}||_2 <= 1 / Im z, so |x - x*| <= ||b - (z - H) x|| / Im z."""
    H, z = small
    b = O.unit(H.n, 9)
    out = O.shifted_cocg(H, z, b, tol=1e-4, max_iter=2000)
    A = H.to_dense()
    for k in range(len(z)):
        xd = _dense_solve(H, z[k], b)
        rt = np.linalg.norm(b - (z[k] * np.eye(H.n) - A) @ out["X"][k])
        assert np.linalg.norm(out["X"][k] - xd) <= rt / z[k].imag * (1 + 1e-9)
        # and the true residual agrees with the recursive one at this accuracy
        assert rt <= 10 * max(out["res"][k], 1e-14)


def test_closed_form_clean_cubic_lattice():
    """Whole pipeline on a clean periodic L^3 lattice: G_00(z) = (1/L^3) sum_k 1/(z - e_k),
    e_k = -2 sum_a cos k_a, k_a = 2 pi m / L (Bloch's theorem)."""
    L = 8
    H = simple_cubic(L, np.zeros(L ** 3))
    z = np.linspace(-7, 7, 16) + 0.05j
    out = O.shifted_cocg(H, z, O.unit(H.n, 0), tol=1e-11, max_iter=3000)
    assert out["ret"] == O.OK
    ka = 2 * np.pi * np.arange(L) / L
    ek = (-2 * (np.cos(ka)[:, None, None] + np.cos(ka)[None, :, None] + np.cos(ka)[None, None, :])).ravel()
    for k in range(len(z)):
        g = np.mean(1.0 / (z[k] - ek))
        assert abs(out["X"][k][0] - g) <= 1e-11 / z[k].imag * 10


@pytest.mark.slow
def test_closed_form_config1_size():
    """Same closed form at the 16^3 size of the cubic workload (zero disorder, eta = 0.01)."""
    p = config1_cubic(disorder=0.0)
    out = O.shifted_cocg(p.H, p.z, O.unit(p.H.n, 0), tol=1e-10, max_iter=3000)
    assert out["ret"] == O.OK
    L = 16
    ka = 2 * np.pi * np.arange(L) / L
    ek = (-2 * (np.cos(ka)[:, None, None] + np.cos(ka)[None, :, None] + np.cos(ka)[None, None, :])).ravel()
    for k in range(len(p.z)):
        g = np.mean(1.0 / (p.z[k] - ek))
        assert abs(out["X"][k][0] - g) <= 1e-10 / p.z[k].imag * 10


def test_spectral_sum_rules():
    """From Sec. 2.1.1 eqs. densityM/gf with f = 1: (1/2 pi i) closed-contour integrals
    of G_jj, z G_jj and z^2 G_jj around the whole spectrum give 1, H_jj and (H^2)_jj."""
    rng = np.random.default_rng(5)
    H = random_sparse_symmetric(30, 0.15, rng)
    lo, hi = O.gershgorin(H)
    c, R = 0.5 * (lo + hi), 0.5 * (hi - lo) + 1.0
    nq = 96
    th = 2 * np.pi * (np.arange(nq) + 0.5) / nq
    zq = c + R * np.exp(1j * th)
    dz = R * np.exp(1j * th) / nq  # (1/2 pi i) dz on the trapezoid rule
    A = H.to_dense()
    A2 = A @ A
    for j in (0, 13, 29):
        out = O.shifted_cocg(H, zq, O.unit(H.n, j), tol=1e-13, max_iter=500)
        g = out["X"][:, j]
        assert abs(np.sum(dz * g) - 1.0) < 1e-10
        assert abs(np.sum(dz * zq * g) - A[j, j]) < 1e-10
        assert abs(np.sum(dz * zq ** 2 * g) - A2[j, j]) < 1e-9


def _gapped_matrix(n, rng):
    """Random sparse symmetric matrix whose spectrum has a clean gap around 0."""
    H = random_sparse_symmetric(n, 0.1, rng)
    A = H.to_dense()
    w, V = np.linalg.eigh(A)
    w = np.where(w < np.median(w), w - 1.0, w + 1.0)
    return w, V


def test_band_energy_and_density_matrix_match_eigendecomposition():
    """Sec. 2.1.1: rho = sum_occ |phi><phi| (eq. densityM-1) equals the contour integral
    of G (eq. densityM at T = 0), and E = Tr[rho H] = sum of occupied eigenvalues."""
    from workloads import diamond

    rng = np.random.default_rng(2)
    H, _ = diamond(1, 1, 1, rng)
    A = H.to_dense()
    w, V = np.linalg.eigh(A)
    mu = 0.5 * (w[15] + w[16])  # half filling, inside the gap between the two middle levels
    # shift the Fermi level to 0 by moving the diagonal (keeps the CSR pattern)
    from workloads import CSR

    vals = H.val.copy()
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    vals[rows == H.col] -= mu
    Hs = CSR(H.n, H.row_ptr, H.col, vals)
    ws = w - mu
    gap = min(abs(ws))
    lo, _ = O.gershgorin(Hs)
    zq, Wq = O.contour(lo - 1.0, 0.0, 128)
    out = O.density_matrix_energy(Hs, zq, Wq, tol=1e-13, max_iter=2000)
    E_exact = np.sum(ws[ws < 0])
    assert gap > 0.05
    assert abs(out["E"] - E_exact) < 1e-8 * max(1.0, abs(E_exact))
    occ = V[:, ws < 0]
    rho_d = occ @ occ.T
    assert np.max(np.abs(out["rho"] - rho_d[rows, H.col])) < 1e-8
    # E = Tr[rho H] over the stored entries
    assert abs(np.sum(out["rho"] * Hs.val) - E_exact) < 1e-8 * max(1.0, abs(E_exact))


def test_band_energy_gradient_dense_and_finite_difference():
    """Derivative of the discrete band energy: dense (G^2)_ab and central differences."""
    from workloads import CSR, diamond

    rng = np.random.default_rng(4)
    H, _ = diamond(1, 1, 1, rng)
    lo, _ = O.gershgorin(H)
    zq, Wq = O.contour(lo - 1.0, 0.0, 48)
    # make sure no eigenvalue sits near the contour's real-axis end mu = 0
    w = np.linalg.eigvalsh(H.to_dense())
    assert np.min(np.abs(w)) > 0.02
    out = O.density_matrix_energy(H, zq, Wq, tol=1e-13, max_iter=3000)
    A = H.to_dense()
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    dense = np.zeros(H.nnz)
    for zk, wk in zip(zq, Wq):
        G = np.linalg.inv(zk * np.eye(H.n) - A)
        dense += np.real(wk * zk * (G @ G)[rows, H.col])
    assert np.max(np.abs(out["grad"] - dense)) < 1e-9 * max(1.0, np.max(np.abs(dense)))
    # central finite differences on a symmetric pair (a, b) and on a diagonal entry
    h = 1e-5
    picks = [k for k in range(H.nnz) if rows[k] < H.col[k]][:3] + [k for k in range(H.nnz) if rows[k] == H.col[k]][:2]
    for k in picks:
        a, b = rows[k], H.col[k]
        mirror = [m for m in range(H.nnz) if rows[m] == b and H.col[m] == a][0]
        Es = []
        for sgn in (+1, -1):
            v = H.val.copy()
            v[k] += sgn * h
            if mirror != k:
                v[mirror] += sgn * h
            Es.append(O.density_matrix_energy(CSR(H.n, H.row_ptr, H.col, v), zq, Wq, tol=1e-13, max_iter=3000)["E"])
        fd = (Es[0] - Es[1]) / (2 * h)
        an = out["grad"][k] + (out["grad"][mirror] if mirror != k else 0.0)
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an))


def test_breakdown_is_reported():
    """b.b = 0 (unconjugated) stops COCG at the first step; the oracle reports breakdown."""
    rng = np.random.default_rng(0)
    H = random_sparse_symmetric(20, 0.2, rng)
    b = O.unit(20, 0) + 1j * O.unit(20, 1)
    out = O.shifted_cocg(H, np.array([0.3 + 0.1j, 1.0 + 0.2j]), b)
    assert out["ret"] == O.EBREAKDOWN
    assert np.all(out["status"] == O.EBREAKDOWN)


def test_non_convergence_is_reported(small):
    H, z = small
    out = O.shifted_cocg(H, z, O.unit(H.n, 1), tol=1e-12, max_iter=1)
    assert out["ret"] == O.ENOCONV
    assert np.all(out["iters"] == 1)


def test_zero_rhs_gives_zero():
    rng = np.random.default_rng(0)
    H = random_sparse_symmetric(10, 0.3, rng)
    out = O.shifted_cocg(H, np.array([0.1 + 0.1j]), np.zeros(10, dtype=complex))
    assert out["ret"] == O.OK and np.all(out["X"] == 0)


def test_freeze_iteration_is_rounding_sensitive():
    """Why tolerance-stopped runs are compared through the residual bound: the oracle on the
    same matrix with its rows permuted (identical mathematics, different summation order)
    freezes some shifts a few iterations apart, while the answers agree to the bound."""
    from workloads import coo_to_csr

    rng = np.random.default_rng(11)
    L = 6
    H = simple_cubic(L, rng.uniform(-1, 1, L ** 3))
    z = np.concatenate([np.linspace(-6, 6, 13) + 0.8j, [0.3 + 3.0j, -2 + 2.5j, 1.0 + 0.7j]])
    b = O.unit(H.n, 0)
    r0 = O.shifted_cocg(H, z, b, tol=1e-10, max_iter=5000, seed_index=13)
    perm = np.random.default_rng(0).permutation(H.n)
    inv = np.argsort(perm)
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    Hp = coo_to_csr(H.n, inv[rows], inv[H.col], H.val)
    r1 = O.shifted_cocg(Hp, z, b[perm], tol=1e-10, max_iter=5000, seed_index=13)
    assert not np.array_equal(r0["iters"], r1["iters"])
    assert np.max(np.abs(r0["iters"] - r1["iters"])) <= 5
    for k in range(len(z)):
        assert abs(r0["X"][k][0] - r1["X"][k][inv[0]]) <= 2 * 20 * 1e-10 / z[k].imag


def test_true_residual_equals_dense_residual():
    """Sec. 3.4 eq. residual: the oracle's true residual ||b - (z - H) x|| / ||b|| against the
    same norm formed from the dense matrix, for complex x, b and shifts on both sides of the
    real axis; with b = 0 the norm is returned unscaled.  Every residual-bound parity check
    uses this routine, so an error in it (a sign of z, a dropped diagonal, a missing square
    root or scale) would loosen those checks; each such mistake fails here."""
    rng = np.random.default_rng(41)
    H = random_sparse_symmetric(40, 0.1, rng, diag_scale=2.0)
    A = H.to_dense()
    I = np.eye(H.n)
    for z in (0.3 + 0.05j, -1.7 + 0.4j, 2.2 - 0.3j, 0.0 + 1.0j):
        x = rng.normal(size=H.n) + 1j * rng.normal(size=H.n)
        b = rng.normal(size=H.n) + 1j * rng.normal(size=H.n)
        dense = np.linalg.norm(b - (z * I - A) @ x) / np.linalg.norm(b)
        assert abs(O.true_residual(H, z, x, b) - dense) <= 1e-13 * dense
        # at the dense solution the residual vanishes to rounding
        xs = np.linalg.solve(z * I - A, b)
        assert O.true_residual(H, z, xs, b) < 1e-13
        # a zero right-hand side: the unscaled norm of (z - H) x
        zero = np.zeros(H.n, dtype=np.complex128)
        ref0 = np.linalg.norm((z * I - A) @ x)
        assert abs(O.true_residual(H, z, x, zero) - ref0) <= 1e-13 * ref0
    # x = 0 gives exactly 1
    b = rng.normal(size=H.n) + 1j * rng.normal(size=H.n)
    assert O.true_residual(H, 0.5 + 0.1j, np.zeros(H.n, dtype=np.complex128), b) == pytest.approx(1.0, abs=1e-15)


def test_cocg_tolerance_stopped_equals_dense_solve(small):
    """Plain COCG stopped at a tolerance (the single-pair reference of the full-size checks):
    the dense residual of its answer is at the tolerance, its recursive residual agrees with
    the dense one, and the answer is within the Sec. 3.4 bound of the dense solve."""
    H, z = small
    A = H.to_dense()
    rng = np.random.default_rng(8)
    b = rng.normal(size=H.n) + 1j * rng.normal(size=H.n)
    tol = 1e-9
    for zk in z:
        out = O.cocg(H, zk, b, tol=tol, max_iter=5000)
        assert out["status"] == O.OK
        rt = np.linalg.norm(b - (zk * np.eye(H.n) - A) @ out["x"]) / np.linalg.norm(b)
        assert rt < 10 * tol
        assert out["res"] < tol and abs(out["res"] - rt) <= 1e-3 * tol + 1e-12
        xd = _dense_solve(H, zk, b)
        assert np.linalg.norm(out["x"] - xd) <= rt * np.linalg.norm(b) / zk.imag * (1 + 1e-9)


def test_switch_log_follows_residual_rule():
    """Sec. 3.3 seed switching, as read here: when the seed's residual falls below the
    tolerance the iteration continues from the still-active shift with the largest residual.
    Checked against plain per-shift COCG (shift invariance makes the shifted iterates equal
    to it in exact arithmetic): at each logged switch the old seed's own COCG has just crossed
    the tolerance (within the few iterations rounding moves a crossing, 6 % + 2), and the new seed is
    the unconverged shift with the largest residual, by a clear margin."""
    rng = np.random.default_rng(68)
    L = 5
    H = simple_cubic(L, rng.uniform(-1, 1, L ** 3))
    A = H.to_dense()
    # ten shifts spread over the band with uneven damping: residual orders cross, so the seed
    # switches twice (after 24 and 55 iterations), each time to a clear largest residual
    z = rng.uniform(-7, 7, 10) + 1j * rng.uniform(0.05, 1.5, 10)
    first = int(np.argmax(z.imag))
    b = O.unit(H.n, 3)
    tol = 1e-8
    out = O.shifted_cocg(H, z, b, tol=tol, max_iter=6000, seed_index=first)
    assert out["ret"] == O.OK and len(out["switches"]) == 2
    n_max = int(out["iters"].max())
    hist = np.zeros((len(z), n_max + 1))
    for k in range(len(z)):
        for m in range(1, n_max + 1):
            out_k = O.cocg(H, z[k], b, fixed_iter=m)
            hist[k, m] = out_k["res"]
        # the recursive residual the stopping rule reads agrees with the dense one at the end
        rt = np.linalg.norm(b - (z[k] * np.eye(H.n) - A) @ out_k["x"]) / np.linalg.norm(b)
        assert abs(rt - hist[k, n_max]) <= 1e-3 * max(rt, tol) + 1e-12
    hist[:, 0] = 1.0
    cross = np.array([int(np.argmax(hist[k] < tol)) if np.any(hist[k] < tol) else n_max + 1 for k in range(len(z))])
    seed = first
    for it, t in out["switches"]:
        n_done = it + 1
        # near the tolerance COCG's residual is irregular, so a rounding-level difference moves
        # a crossing by a few iterations (the same allowance as the GPU comparisons)
        slack = 0.06 * n_done + 2
        assert abs(cross[seed] - n_done) <= slack, (seed, cross[seed], n_done)
        active = [k for k in range(len(z)) if k != seed and cross[k] > n_done + slack]
        assert t in active
        others = [hist[k, n_done] for k in active if k != t]
        assert hist[t, n_done] > 1.5 * max(others), (t, hist[t, n_done], max(others))
        seed = t
    assert out["final_seed"] == seed
    # every shift's freeze iteration is its own crossing, up to the same allowance
    assert np.all(np.abs(out["iters"] - cross) <= 0.06 * cross + 2)
