"""Python face of the shifted-COCG oracle (plain FP64 CPU reference).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module.  It shares no code with the GPU library.

Layers:
  * ``scocg_oracle.c`` (loaded with ctypes): plain COCG and shifted COCG with
    seed switching (Sec. 3.3), the residual check (Sec. 3.4).
  * this file: Green's-function extraction G_ij(z) = [(z - H)^{-1}]_ij
    (Sec. 2.1.1 eq. gf), the density matrix from a contour integral of G
    (Sec. 2.1.1 eq. densityM at zero temperature) and the band energy
    Tr[rho H] (Sec. 2.1.1, <X> = Tr[rho X] with X = H), plus the exact
    derivative of that discrete band energy with respect to the stored entries
    of H.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scocg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EBREAKDOWN, ENOCONV = 0, 4, 5


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP over the shift loop)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("seed_index", ctypes.c_int),
        ("switching", ctypes.c_int),
        ("fixed_iter", ctypes.c_int),
        ("force_switch_iter", ctypes.c_int),
        ("force_switch_to", ctypes.c_int),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        _lib.oracle_cocg.argtypes = [i64, P, P, P, ctypes.c_double, ctypes.c_double, P, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.oracle_cocg.restype = ctypes.c_int
        _lib.oracle_shifted_cocg.argtypes = [i64, P, P, P, i64, P, P, ctypes.POINTER(_Opts), P, P, P, P, P, P, P,
                                             ctypes.c_int, P, P, P]
        _lib.oracle_shifted_cocg.restype = ctypes.c_int
        _lib.oracle_default_seed.argtypes = [i64, P, P, P, i64, P]
        _lib.oracle_default_seed.restype = ctypes.c_int
        _lib.oracle_true_residual.argtypes = [i64, P, P, P, ctypes.c_double, ctypes.c_double, P, P]
        _lib.oracle_true_residual.restype = ctypes.c_double
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_args(H):
    rp = np.ascontiguousarray(H.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(H.col, dtype=np.int64)
    v = np.ascontiguousarray(H.val, dtype=np.float64)
    return rp, ci, v


def cocg(H, z: complex, b: np.ndarray, tol: float = 1e-12, max_iter: int = 10000, fixed_iter: int = 0):
    """Plain COCG for one shift (the per-shift reference, no shift recurrences)."""
    lib = _load()
    rp, ci, v = _csr_args(H)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros(H.n, dtype=np.complex128)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0)
    st = lib.oracle_cocg(H.n, _ptr(rp), _ptr(ci), _ptr(v), float(np.real(z)), float(np.imag(z)), _ptr(b), tol,
                         max_iter, fixed_iter, _ptr(x), ctypes.byref(it), ctypes.byref(res))
    return dict(x=x, iters=it.value, status=st, res=res.value)


def default_seed(H, z) -> int:
    lib = _load()
    rp, ci, v = _csr_args(H)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    return lib.oracle_default_seed(H.n, _ptr(rp), _ptr(ci), _ptr(v), len(z), _ptr(z))


def shifted_cocg(H, z, b, tol: float = 1e-8, max_iter: int = 3000, seed_index: int = -1, switching: bool = True,
                 fixed_iter: int = 0, force_switch=None, max_log: int = 4096):
    """Shifted COCG with seed switching for one RHS; returns a dict of numpy results."""
    lib = _load()
    rp, ci, v = _csr_args(H)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    m, n = len(z), H.n
    o = _Opts(tol, max_iter, seed_index, int(switching), fixed_iter,
              -1 if force_switch is None else force_switch[0], -1 if force_switch is None else force_switch[1])
    X = np.zeros((m, n), dtype=np.complex128)
    iters = np.zeros(m, dtype=np.int32)
    status = np.zeros(m, dtype=np.int32)
    res = np.zeros(m)
    r = np.zeros(n, dtype=np.complex128)
    pi = np.zeros(m, dtype=np.complex128)
    log = np.zeros(2 * max_log, dtype=np.int32)
    nsw = ctypes.c_int(0)
    fseed = ctypes.c_int(0)
    tot = ctypes.c_int(0)
    ret = lib.oracle_shifted_cocg(n, _ptr(rp), _ptr(ci), _ptr(v), m, _ptr(z), _ptr(b), ctypes.byref(o), _ptr(X),
                                  _ptr(iters), _ptr(status), _ptr(res), _ptr(r), _ptr(pi), _ptr(log), max_log,
                                  ctypes.byref(nsw), ctypes.byref(fseed), ctypes.byref(tot))
    k = min(nsw.value, max_log)
    return dict(X=X, iters=iters, status=status, res=res, r=r, pi=pi, ret=ret,
                switches=[(int(log[2 * i]), int(log[2 * i + 1])) for i in range(k)], final_seed=fseed.value,
                total_iters=tot.value)


def true_residual(H, z: complex, x, b) -> float:
    lib = _load()
    rp, ci, v = _csr_args(H)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    return lib.oracle_true_residual(H.n, _ptr(rp), _ptr(ci), _ptr(v), float(np.real(z)), float(np.imag(z)), _ptr(x),
                                    _ptr(b))


def unit(n: int, j: int) -> np.ndarray:
    e = np.zeros(n, dtype=np.complex128)
    e[j] = 1.0
    return e


def greens_diag(H, z, rhs_idx, **kw):
    """G_jj(z_k) = [(z_k - H)^{-1}]_jj for j in rhs_idx (Sec. 2.1.1 eq. gf); returns G[M, K] and the runs."""
    z = np.asarray(z, dtype=np.complex128)
    G = np.zeros((len(z), len(rhs_idx)), dtype=np.complex128)
    runs = []
    for c, j in enumerate(rhs_idx):
        out = shifted_cocg(H, z, unit(H.n, int(j)), **kw)
        G[:, c] = out["X"][:, int(j)]
        runs.append(out)
    return G, runs


def gershgorin(H):
    """Gershgorin interval [lo, hi] containing the spectrum of H."""
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    d = np.zeros(H.n)
    off = np.zeros(H.n)
    isd = rows == H.col
    d[rows[isd]] = H.val[isd]
    np.add.at(off, rows[~isd], np.abs(H.val[~isd]))
    return float(np.min(d - off)), float(np.max(d + off))


def contour(e_lo: float, mu: float, n_quad: int):
    """Nodes and complex weights for rho = (1/2 pi i) closed-contour integral of G dz.

    The contour is the circle through e_lo and mu (centre c, radius R).  For a
    real-symmetric H, G(conj z) = conj G(z), so the closed integral is
    (1/pi) Re of the integral over the upper half, theta in (0, pi), with
    dz = i R e^{i theta} d theta.  Gauss-Legendre on theta gives
        rho ~= Re sum_k W_k G(z_k),   W_k = w_k R e^{i theta_k} / pi.
    Returns (z[n_quad], W[n_quad]) complex.
    """
    c = 0.5 * (e_lo + mu)
    R = 0.5 * (mu - e_lo)
    x, w = np.polynomial.legendre.leggauss(n_quad)
    theta = 0.5 * np.pi * (x + 1.0)
    wt = 0.5 * np.pi * w
    e = np.exp(1j * theta)
    return c + R * e, wt * R * e / np.pi


def density_matrix_energy(H, z, W, rhs_idx=None, want_residuals=False, **kw):
    """Density matrix on the stored pattern of H and the band energy E = Tr[rho H].

    rho_ab = Re sum_k W_k G_ab(z_k) for every stored (a, b) (Sec. 2.1.1: only the
    entries of rho where H is non-zero are needed).  G_ab(z_k) = x_{k,b}[a] with
    x_{k,b} = (z_k - H)^{-1} e_b.  rhs_idx restricts the columns b that are
    accumulated (default: all).  Also returns dE/dH_ab, the exact derivative of
    the discrete band energy E = Re sum_k W_k z_k Tr G(z_k):
        dE/dH_ab = Re sum_k W_k z_k (G_k G_k)_ab = Re sum_k W_k z_k sum_j x_kj[a] x_kj[b].
    want_residuals adds res_true[len(rhs_idx), M], the true residual of every solve
    (Sec. 3.4), from which callers bound the error of these sums.
    """
    n = H.n
    z = np.asarray(z, dtype=np.complex128)
    W = np.asarray(W, dtype=np.complex128)
    rhs_idx = np.arange(n) if rhs_idx is None else np.asarray(rhs_idx)
    rows = np.repeat(np.arange(n), np.diff(H.row_ptr))
    cols = H.col
    rho = np.zeros(H.nnz)
    grad = np.zeros(H.nnz)
    E = 0.0
    in_set = np.zeros(n, dtype=bool)
    in_set[rhs_idx] = True
    res_true = np.zeros((len(rhs_idx), len(z))) if want_residuals else None
    for c, j in enumerate(rhs_idx):
        out = shifted_cocg(H, z, unit(n, int(j)), **kw)
        X = out["X"]  # [M, n]: column j of G(z_k)
        if want_residuals:
            for k in range(len(z)):
                res_true[c, k] = true_residual(H, z[k], X[k], unit(n, int(j)))
        # rho_ab for entries in column b = j: G_ab = X[k, a]
        sel = cols == j
        rho[sel] += np.real(W @ X[:, rows[sel]])
        E += float(np.real(np.sum(W * z * X[:, j])))
        # (G^2)_ab accumulates x_kj[a] x_kj[b] over all columns j
        grad += np.real((W * z) @ (X[:, rows] * X[:, cols]))
    out = dict(rho=rho, E=E, grad=grad)
    if want_residuals:
        out["res_true"] = res_true
    return out
