"""PyTorch-facing binding of the shifted-COCG library.

PyTorch provides device memory and the stream; every computation runs in
libscocg.so (HIP kernels for gfx950).  Function names follow the C ABI.
"""

import ctypes

import numpy as np
import torch

from . import _capi as C


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("the shifted-COCG library needs a HIP device; none is visible")


def _device(device):
    """The device for outputs: a HIP device (the library writes through device pointers)."""
    dev = torch.device(device) if device is not None else torch.device("cuda")
    if dev.type != "cuda":
        raise ValueError("outputs must live on a HIP device")
    return dev


def _check_dev(t: torch.Tensor, dtype, numel, name):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor of {numel} elements")


def options(tol=1e-8, max_iter=3000, precision="fp64", seed_index=-1, seed_switching=True, fixed_iter=0, block=0,
            shifts_per_wg=0, check_true=False, keep_tape=False, no_graph=False, refine=0, window=0,
            schedule="auto", update_form="auto") -> C.Opts:
    o = C.Opts()
    C.load().scocg_default_opts(ctypes.byref(o))
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.precision = {"fp64": 0, "fp32": 1, 0: 0, 1: 1}[precision]
    o.seed_index = int(seed_index)
    o.seed_switching = int(bool(seed_switching))
    o.fixed_iter = int(fixed_iter)
    o.block = int(block)
    o.shifts_per_wg = int(shifts_per_wg)
    o.check_true = int(bool(check_true))
    o.keep_tape = int(bool(keep_tape))
    o.no_graph = int(bool(no_graph))
    o.refine = int(refine)
    o.window = int(window)
    o.schedule = {"auto": 0, "serial": 1, "overlap": 2, 0: 0, 1: 1, 2: 2}[schedule]
    o.update_form = {"auto": 0, "step": 1, "expanded": 2, 0: 0, 1: 1, 2: 2}[update_form]
    return o


def csr_validate(row_ptr, col, val) -> None:
    """Host-side check of a CSR matrix (shape, ordering, finiteness, exact symmetry)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col, dtype=np.int64)
    v = np.ascontiguousarray(val, dtype=np.float64)
    n = len(rp) - 1
    C.check(C.load().scocg_csr_validate(n, len(ci), rp.ctypes.data, ci.ctypes.data, v.ctypes.data))


class Hamiltonian:
    """A real-symmetric sparse H uploaded to the current device (csr_upload)."""

    def __init__(self, row_ptr, col, val, validate=True):
        _require_gpu()
        lib = C.load()
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col, dtype=np.int64)
        v = np.ascontiguousarray(val, dtype=np.float64)
        self.n = len(rp) - 1
        self.nnz = len(ci)
        self.row_ptr, self.col = rp, ci
        h = ctypes.c_void_p()
        C.check(lib.csr_upload(self.n, self.nnz, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, int(validate),
                               _stream_ptr(), ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_csr(cls, H, validate=True):
        return cls(H.row_ptr, H.col, H.val, validate=validate)

    @classmethod
    def hubbard(cls, L, n_up, n_dn, t=1.0, U=4.0, V=1.0):
        """Matrix-free extended Hubbard ring (hubbard_upload): the sector Hamiltonian applied
        from per-species hopping tables instead of a stored matrix."""
        _require_gpu()
        lib = C.load()
        self = cls.__new__(cls)
        h = ctypes.c_void_p()
        C.check(lib.hubbard_upload(int(L), int(n_up), int(n_dn), float(t), float(U), float(V), _stream_ptr(),
                                   ctypes.byref(h)))
        self._h = h
        self.n = int(lib.csr_n(h))
        self.nnz = int(lib.csr_nnz(h))
        self.row_ptr = self.col = None
        return self

    @property
    def handle(self):
        return self._h

    def update_values(self, val):
        v = np.ascontiguousarray(val, dtype=np.float64)
        if len(v) != self.nnz:
            raise ValueError("value array has the wrong length")
        C.check(C.load().csr_update_values(self._h, v.ctypes.data, _stream_ptr()))

    def close(self):
        if getattr(self, "_h", None):
            C.load().csr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tape:
    """Solutions kept by a solve for backward().  The library keeps the matrix the tape was
    recorded on alive until the tape is freed; the tape also holds the Python Hamiltonian."""

    def __init__(self, h, kind, n_shift, n_rhs, nnz, hamiltonian=None):
        self._h = h
        self.hamiltonian = hamiltonian
        self.kind = kind
        self.nnz = nnz
        self.n_shift = n_shift
        self.n_rhs = n_rhs

    def close(self):
        if getattr(self, "_h", None):
            C.load().tape_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _z_host(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    return z, z.ctypes.data


def _report(rep, n_rhs, n_shift):
    a = np.ctypeslib.as_array(rep, shape=(n_rhs * n_shift,))
    return dict(iters=np.array(a["iters"]).reshape(n_rhs, n_shift),
                status=np.array(a["status"]).reshape(n_rhs, n_shift),
                res=np.array(a["rel_res_recursive"]).reshape(n_rhs, n_shift),
                res_true=np.array(a["rel_res_true"]).reshape(n_rhs, n_shift))


def last_timing() -> dict:
    t = C.Timing()
    C.load().scocg_last_timing(ctypes.byref(t))
    return {f: getattr(t, f) for f, _ in C.Timing._fields_}


def last_switches(n_rhs: int) -> list:
    """Seed switches of the last solve on this thread: for each right-hand side, the list of
    (iterations completed when the old seed converged, new seed shift)."""
    lib = C.load()
    out = []
    for j in range(int(n_rhs)):
        c = lib.scocg_last_switches(j, None, 0)
        if c < 0:
            raise C.ScocgError(C.EINVAL, lib.scocg_last_error().decode())
        buf = (ctypes.c_int32 * (2 * max(c, 1)))()
        lib.scocg_last_switches(j, buf, c)
        out.append([(int(buf[2 * e]), int(buf[2 * e + 1])) for e in range(c)])
    return out


def set_profiling(on: bool) -> None:
    C.load().scocg_set_profiling(int(bool(on)))


def _allowed(allow_noconv, allow_breakdown):
    a = [C.OK]
    if allow_noconv:
        a.append(C.ENOCONV)
    if allow_breakdown:
        a.append(C.EBREAKDOWN)
    return tuple(a)


def shifted_cocg_solve(H: Hamiltonian, z, B: torch.Tensor, out: torch.Tensor = None, allow_noconv=True,
                       allow_breakdown=False, **opts):
    """Solve (z_k - H) X[j, k] = B[j] for every shift k and right-hand side j.

    B is a complex128 device tensor [n_rhs, n].  Returns (X [n_rhs, n_shift, n],
    report dict, tape or None, status code).
    """
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    if B.dtype != torch.complex128 or not B.is_cuda or B.dim() != 2 or B.shape[1] != H.n:
        raise ValueError("B must be a complex128 device tensor of shape [n_rhs, n]")
    B = B.contiguous()
    K, M = B.shape[0], len(zh)
    if out is None:
        out = torch.empty((K, M, H.n), dtype=torch.complex128, device=B.device)
    _check_dev(out, torch.complex128, K * M * H.n, "out")
    o = options(**opts)
    rep = (C.PairReport * (K * M))()
    tape = ctypes.c_void_p()
    rc = lib.shifted_cocg_solve(H.handle, M, zp, K, B.data_ptr(), ctypes.byref(o), out.data_ptr(), rep,
                                ctypes.byref(tape) if o.keep_tape else None, _stream_ptr())
    C.check(rc, allow=_allowed(allow_noconv, allow_breakdown))
    t = Tape(tape, "solve", M, K, H.nnz, H) if o.keep_tape and tape.value else None
    return out, _report(rep, K, M), t, rc


def greens_diag(H: Hamiltonian, z, rhs_idx, allow_noconv=True, allow_breakdown=False, device=None, **opts):
    """G_jj(z_k) for unit right-hand sides e_j (j in rhs_idx); returns (G [n_shift, n_rhs], report, tape, rc)."""
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    idx = np.ascontiguousarray(rhs_idx, dtype=np.int64)
    K, M = len(idx), len(zh)
    G = torch.empty((M, K), dtype=torch.complex128, device=_device(device))
    o = options(**opts)
    rep = (C.PairReport * (K * M))()
    tape = ctypes.c_void_p()
    rc = lib.greens_diag(H.handle, M, zp, K, idx.ctypes.data, ctypes.byref(o), G.data_ptr(), rep,
                         ctypes.byref(tape) if o.keep_tape else None, _stream_ptr())
    C.check(rc, allow=_allowed(allow_noconv, allow_breakdown))
    t = Tape(tape, "greens", M, K, H.nnz, H) if o.keep_tape and tape.value else None
    return G, _report(rep, K, M), t, rc


def greens_diag_noalloc(H: Hamiltonian, z, rhs_idx, G: torch.Tensor = None, allow_noconv=True, allow_breakdown=False,
                        **opts):
    """greens_diag whose work buffers live in the library's fixed device array (no device
    allocation inside the call).  G, if given, is the [n_shift, n_rhs] complex128 output (allocate
    it beforehand to keep the whole call allocation-free).  Returns (G, report, rc)."""
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    idx = np.ascontiguousarray(rhs_idx, dtype=np.int64)
    K, M = len(idx), len(zh)
    if G is None:
        G = torch.empty((M, K), dtype=torch.complex128, device="cuda")
    _check_dev(G, torch.complex128, M * K, "G")
    o = options(**opts)
    rep = (C.PairReport * (K * M))()
    rc = lib.greens_diag_noalloc(H.handle, M, zp, K, idx.ctypes.data, ctypes.byref(o), G.data_ptr(), rep,
                                 _stream_ptr())
    C.check(rc, allow=_allowed(allow_noconv, allow_breakdown))
    return G, _report(rep, K, M), rc


def krylov_greens_diag(H: Hamiltonian, z, rhs_idx, nu: int, device=None):
    """Local Green's functions G_jj(z_k) by Krylov-subspace diagonalization (nu steps of the
    three-term recurrence from each unit vector e_j, then the reduced tridiagonal Hamiltonian).

    Returns (G [n_shift, n_rhs] complex128, ab [n_rhs, 2, nu] float64 with the diagonal a and
    the off-diagonal b of each reduced Hamiltonian, dim [n_rhs] int32 subspace dimensions)."""
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    idx = np.ascontiguousarray(rhs_idx, dtype=np.int64)
    K, M = len(idx), len(zh)
    dev = _device(device)
    G = torch.empty((M, K), dtype=torch.complex128, device=dev)
    ab = torch.zeros((K, 2, int(nu)), dtype=torch.float64, device=dev)
    dim = np.zeros(K, dtype=np.int32)
    rc = lib.krylov_greens_diag(H.handle, M, zp, K, idx.ctypes.data, int(nu), G.data_ptr(), ab.data_ptr(),
                                dim.ctypes.data, _stream_ptr())
    C.check(rc)
    return G, ab, dim


def krylov_greens_vec(H: Hamiltonian, z, b, nu: int, device=None):
    """<b|(z_k - H)^{-1}|b> for a real start vector b by Krylov-subspace diagonalization (nu
    steps of the three-term recurrence from b / |b|, then the continued fraction).  Returns
    (G [n_shift] complex128, ab [2, nu] float64, subspace dimension)."""
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    dev = _device(device)
    bt = torch.as_tensor(b)
    if bt.is_complex():
        if bool(torch.any(bt.imag != 0)):
            raise ValueError("the start vector must be real")
        bt = bt.real
    bt = bt.to(device=dev, dtype=torch.float64).contiguous()
    if bt.numel() != H.n:
        raise ValueError("b must have one entry per row")
    M = len(zh)
    G = torch.empty(M, dtype=torch.complex128, device=dev)
    ab = torch.zeros((2, int(nu)), dtype=torch.float64, device=dev)
    dim = ctypes.c_int32()
    rc = lib.krylov_greens_vec(H.handle, M, zp, bt.data_ptr(), int(nu), G.data_ptr(), ab.data_ptr(),
                               ctypes.byref(dim), _stream_ptr())
    C.check(rc)
    return G, ab, dim.value


def ground_state(H: Hamiltonian, x0, nu: int = 200, tol: float = 1e-10, max_sweeps: int = 50, device=None,
                 allow_noconv=False):
    """Lowest eigenpair of H: an estimate from nu steps of the three-term recurrence started at
    x0, refined by inverse iteration with one-shift CG solves.  Returns (psi [n] complex128,
    E0, E1 estimate, residual ||H psi - E0 psi||, sweeps).  A residual still above tol after
    max_sweeps raises, unless allow_noconv (then the result is returned as it stands)."""
    _require_gpu()
    lib = C.load()
    dev = _device(device)
    x = torch.as_tensor(x0, dtype=torch.float64).to(dev).contiguous()
    if x.numel() != H.n:
        raise ValueError("x0 must have one entry per row")
    psi = torch.empty(H.n, dtype=torch.complex128, device=dev)
    E = (ctypes.c_double * 2)()
    res = ctypes.c_double()
    sweeps = ctypes.c_int32()
    rc = lib.ground_state(H.handle, x.data_ptr(), int(nu), float(tol), int(max_sweeps), psi.data_ptr(), E,
                          ctypes.byref(res), ctypes.byref(sweeps), _stream_ptr())
    C.check(rc, allow=(C.OK, C.ENOCONV) if allow_noconv else (C.OK,))
    return psi, E[0], E[1], res.value, sweeps.value


def hubbard_fermion_op(L: int, n_up: int, n_dn: int, site: int, spin: int, create: bool, x: torch.Tensor):
    """c_{site,spin} x or c+_{site,spin} x (spin 0 = up) from the sector (L, n_up, n_dn) of the
    Hubbard ring to its neighbour sector; returns (y complex128, (n_up', n_dn'))."""
    _require_gpu()
    from math import comb

    lib = C.load()
    d = 1 if create else -1
    tu, td = (n_up + d, n_dn) if spin == 0 else (n_up, n_dn + d)
    if not (0 <= tu <= L and 0 <= td <= L):
        raise ValueError("the target sector does not exist")
    if x.dtype != torch.complex128 or not x.is_cuda or x.numel() != comb(L, n_up) * comb(L, n_dn):
        raise ValueError("x must be a complex128 device vector of the source sector")
    x = x.contiguous()
    y = torch.empty(comb(L, tu) * comb(L, td), dtype=torch.complex128, device=x.device)
    rc = lib.hubbard_fermion_op(int(L), int(n_up), int(n_dn), int(site), int(spin), int(bool(create)), x.data_ptr(),
                                y.data_ptr(), _stream_ptr())
    C.check(rc)
    return y, (tu, td)


def greens_proj(H: Hamiltonian, z, B: torch.Tensor, W: torch.Tensor = None, allow_noconv=True, allow_breakdown=False,
                **opts):
    """<w_j|(z_k - H)^{-1}|b_j> (bilinear) for the rows b_j of B and w_j of W (default W = B),
    every shift carried by scalars; full directions only for `window` seed candidates.
    Returns (G [n_shift, n_rhs] complex128, report dict, timing dict, status)."""
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    W = B if W is None else W
    for T in (B, W):
        if T.dtype != torch.complex128 or not T.is_cuda or T.dim() != 2 or T.shape[1] != H.n:
            raise ValueError("B and W must be complex128 device tensors of shape [n_rhs, n]")
    if W.shape != B.shape or W.device != B.device:
        raise ValueError("W must match B")
    B, W = B.contiguous(), W.contiguous()
    K, M = B.shape[0], len(zh)
    o = options(**opts)
    G = torch.empty((M, K), dtype=torch.complex128, device=B.device)
    rep = (C.PairReport * (K * M))()
    rc = lib.greens_proj(H.handle, M, zp, K, B.data_ptr(), W.data_ptr(), ctypes.byref(o), G.data_ptr(), rep,
                         _stream_ptr())
    C.check(rc, allow=_allowed(allow_noconv, allow_breakdown))
    return G, _report(rep, K, M), last_timing(), rc


def greens_diag_batched(Hs, z, rhs_lists, allow_noconv=True, allow_breakdown=False, **opts):
    """G_jj(z_k) for several Hamiltonians of different sizes in one solve.

    Hs: list of Hamiltonian; rhs_lists: per problem, the row indices j of its unit
    right-hand sides.  Returns (list of G_q [n_shift, len(rhs_lists[q])], list of reports, rc).
    """
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    counts = np.array([len(r) for r in rhs_lists], dtype=np.int64)
    idx = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=np.int64) for r in rhs_lists]))
    handles = (ctypes.c_void_p * len(Hs))(*[H.handle.value for H in Hs])
    K, M = int(counts.sum()), len(zh)
    G = torch.empty((M, K), dtype=torch.complex128, device=torch.device("cuda"))
    o = options(**opts)
    rep = (C.PairReport * (K * M))()
    rc = lib.greens_diag_batched(len(Hs), handles, counts.ctypes.data, idx.ctypes.data, M, zp, ctypes.byref(o),
                                 G.data_ptr(), rep, _stream_ptr())
    C.check(rc, allow=_allowed(allow_noconv, allow_breakdown))
    full = _report(rep, K, M)
    bounds = np.concatenate([[0], np.cumsum(counts)])
    Gs = [G[:, bounds[q]:bounds[q + 1]] for q in range(len(Hs))]
    reps = [{k: v[bounds[q]:bounds[q + 1]] for k, v in full.items()} for q in range(len(Hs))]
    return Gs, reps, rc


def greens_diag_waves(Hs, z, rhs_lists, max_bytes=64e9, **opts):
    """greens_diag_batched over waves of problems whose stored directions fit in max_bytes."""
    esz = 8 if opts.get("precision", "fp64") in ("fp32", 1) else 16
    M = len(z) if not opts.get("window") else min(len(z), int(opts["window"]))
    waves, cur, cur_bytes = [], [], 0.0
    for q, (H, r) in enumerate(zip(Hs, rhs_lists)):
        b = esz * M * len(r) * H.n
        if cur and cur_bytes + b > max_bytes:
            waves.append(cur)
            cur, cur_bytes = [], 0.0
        cur.append(q)
        cur_bytes += b
    if cur:
        waves.append(cur)
    Gs, reps, rcs = [None] * len(Hs), [None] * len(Hs), []
    for w in waves:
        g, rp, rc = greens_diag_batched([Hs[q] for q in w], z, [rhs_lists[q] for q in w], **opts)
        for i, q in enumerate(w):
            Gs[q], reps[q] = g[i], rp[i]
        rcs.append(rc)
    return Gs, reps, max(rcs), waves


def contour(e_lo: float, mu: float, n_quad: int):
    """Zero-temperature contour nodes z_q and weights w_q (rho = Re sum_q w_q G(z_q))."""
    z = np.zeros(n_quad, dtype=np.complex128)
    w = np.zeros(n_quad, dtype=np.complex128)
    C.check(C.load().scocg_contour(float(e_lo), float(mu), int(n_quad), z.ctypes.data, w.ctypes.data))
    return z, w


def density_matrix_energy(H: Hamiltonian, z, w, rhs_idx=None, want_rho=True, want_grad=False, rhs_batch=0,
                          allow_noconv=True, **opts):
    """rho on H's stored entries, band energy E and dE/dH_ab for the columns in rhs_idx."""
    _require_gpu()
    lib = C.load()
    zh, zp = _z_host(z)
    wh, wp = _z_host(w)
    if len(wh) != len(zh):
        raise ValueError("z and w must have the same length")
    idx = np.ascontiguousarray(np.arange(H.n) if rhs_idx is None else rhs_idx, dtype=np.int64)
    dev = torch.device("cuda")
    rho = torch.zeros(H.nnz, dtype=torch.float64, device=dev) if want_rho else None
    grad = torch.zeros(H.nnz, dtype=torch.float64, device=dev) if want_grad else None
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    o = options(**opts)
    rc = lib.density_matrix_energy(H.handle, len(zh), zp, wp, len(idx), idx.ctypes.data, ctypes.byref(o),
                                   int(rhs_batch), rho.data_ptr() if rho is not None else None, E.data_ptr(),
                                   grad.data_ptr() if grad is not None else None, _stream_ptr())
    C.check(rc, allow=(C.OK, C.ENOCONV) if allow_noconv else (C.OK,))
    return dict(rho=rho, E=E, grad=grad, rc=rc)


def backward(tape: Tape, grad_G: torch.Tensor, grad_val: torch.Tensor = None) -> torch.Tensor:
    """dL/dH per stored CSR entry from dL/dG ([n_shift, n_rhs] complex128, PyTorch's convention
    g = dL/dRe G + i dL/dIm G).  Accumulates into grad_val if given."""
    _require_gpu()
    if tape is None or tape._h is None:
        raise ValueError("no tape")
    g = grad_G.to(device=_device(grad_G.device if grad_G.is_cuda else None), dtype=torch.complex128).contiguous()
    if tuple(g.shape) != (tape.n_shift, tape.n_rhs):
        raise ValueError("grad_G must have shape [n_shift, n_rhs]")
    if grad_val is None:
        grad_val = torch.zeros(tape.nnz, dtype=torch.float64, device=g.device)
    _check_dev(grad_val, torch.float64, tape.nnz, "grad_val")
    C.check(C.load().backward(tape._h, g.data_ptr(), grad_val.data_ptr(), _stream_ptr()))
    return grad_val
