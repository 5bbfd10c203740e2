"""Krylov-subspace diagonalization reference (plain FP64 CPU), for the method of Sec. 3.2.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg use this
module.  It shares no code with the GPU library.

The method (Sec. 3.2, eq. Ham_in_KS): the Krylov subspace K_nu(H, |j>) gets an orthonormal
basis {|K_n>} from the three-term (Lanczos) recurrence; the reduced Hamiltonian
{<K_n|H|K_m>} is then tridiagonal, and diagonalizing it gives approximate eigenpairs
(e_a, |w_a>) in the subspace, from which the local Green's function follows as
G_jj(z) = sum_a |<j|w_a>|^2 / (z - e_a) (Sec. 2.1.1 eq. gf in the eigenbasis).

Readings (the paper states the method, not its recurrence):
  * start vector |K_1> = |j> (unit vector, real: every basis vector stays real for real H);
  * recurrence, per step n = 1 .. nu:  w = H K_n - b_n K_{n-1};  a_n = <K_n|w>;
    w <- w - a_n K_n;  b_{n+1} = ||w||;  K_{n+1} = w / b_{n+1}  (b_1 = 0);
  * the reduced Hamiltonian is the nu x nu tridiagonal T with diagonal a_1..a_nu and
    off-diagonal b_2..b_nu; b_{nu+1} is the norm of what the subspace leaves out;
  * an invariant subspace ends the recurrence early: if b_{n+1} <= 1e-12 (|a_n| + b_n) the
    subspace has dimension n.
"""

import numpy as np

STOP_REL = 1e-12


def matvec(H, v):
    """y = H v for the CSR matrix H (row_ptr, col, val)."""
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    return np.bincount(rows, weights=H.val * v[H.col], minlength=H.n)


def lanczos(H, j: int, nu: int):
    """Coefficients of the Krylov basis of |j>: a[0..m), b[0..m) with b[n] = b_{n+2} in the
    1-based notation above (b[n] couples K_{n+1} and K_{n+2}; b[m-1] is the leftover norm),
    m <= nu the subspace dimension reached."""
    v = np.zeros(H.n)
    v[j] = 1.0
    return lanczos_from(H, v, nu)


def lanczos_from(H, v, nu: int):
    """The same recurrence from a real unit start vector |K_1> = v."""
    v_prev = np.zeros(H.n)
    v = np.asarray(v, dtype=float).copy()
    b_n = 0.0
    a, b = [], []
    for n in range(nu):
        w = matvec(H, v) - b_n * v_prev
        a_n = float(v @ w)
        w = w - a_n * v
        b_next = float(np.sqrt(w @ w))
        a.append(a_n)
        b.append(b_next)
        if n == nu - 1 or b_next <= STOP_REL * (abs(a_n) + b_n):
            break
        v_prev, v = v, w / b_next
        b_n = b_next
    return np.array(a), np.array(b)


def reduced_hamiltonian(a, b):
    """The tridiagonal {<K_n|H|K_m>} of the subspace (eq. Ham_in_KS)."""
    m = len(a)
    return np.diag(a) + np.diag(b[: m - 1], 1) + np.diag(b[: m - 1], -1)


def greens_from_subspace(a, b, z):
    """G_jj(z) = sum_a |<j|w_a>|^2 / (z - e_a) from the eigenpairs of the reduced
    Hamiltonian; <j|w_a> is the first component of its eigenvector (|j> = |K_1>)."""
    e, U = np.linalg.eigh(reduced_hamiltonian(a, b))
    w = U[0, :] ** 2
    z = np.atleast_1d(np.asarray(z, dtype=complex))
    return (w[None, :] / (z[:, None] - e[None, :])).sum(axis=1)


def krylov_greens_diag(H, z, rhs_idx, nu: int):
    """G[k, r] = G_{j_r j_r}(z_k) in the nu-dimensional Krylov subspace of each |j_r>."""
    cols = []
    for j in rhs_idx:
        a, b = lanczos(H, int(j), nu)
        cols.append(greens_from_subspace(a, b, z))
    return np.stack(cols, axis=1)


def krylov_greens_vec(H, z, b, nu: int):
    """<b|(z - H)^{-1}|b> in the nu-dimensional Krylov subspace of a real start vector b:
    |b|^2 times the subspace Green's function of b / |b| (the method of Sec. 3.2 with the
    start vector b instead of a unit vector)."""
    b = np.asarray(b, dtype=float)
    nb2 = float(b @ b)
    a, c = lanczos_from(H, b / np.sqrt(nb2), nu)
    return nb2 * greens_from_subspace(a, c, z)
