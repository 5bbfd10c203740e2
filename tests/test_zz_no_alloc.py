"""The allocation-free greens_diag entry point against greens_diag, through the C ABI.

greens_diag_noalloc runs the same kernels on buffers carved from the library's fixed device
array, so its Green's functions and reports must equal greens_diag's bit for bit: checked on two
calls in a row (the second smaller, with another precision and block length, so it runs on what
the first left in the array), and an oversized request is refused before any work.
"""

import ctypes

import numpy as np
import pytest

from workloads import simple_cubic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _noalloc(lib, C, H, z, idx, o):
    zh = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    K, M = len(idx), len(zh)
    G = torch.empty((M, K), dtype=torch.complex128, device="cuda")
    rep = (C.PairReport * (K * M))()
    rc = lib.greens_diag_noalloc(H.handle, M, zh.ctypes.data, K, idx.ctypes.data, ctypes.byref(o), G.data_ptr(), rep,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    a = np.ctypeslib.as_array(rep, shape=(K * M,))
    return rc, G.cpu().numpy(), {f: np.array(a[f]).reshape(K, M) for f in ("iters", "status", "rel_res_recursive")}


@pytest.mark.parametrize("first", [True, False])
def test_noalloc_equals_greens_diag_two_calls(first):
    import paper_0802_0748_amd as S
    from paper_0802_0748_amd import _capi as C

    lib = C.load()
    rng = np.random.default_rng(31)
    cases = [
        # larger call first: 512 rows, 3 unit right-hand sides, 16 shifts, FP64, blocks of 48
        dict(L=8, idx=[0, 77, 511], M=16, opts=dict(tol=1e-10, max_iter=6000)),
        # then a smaller one: 216 rows, 2 right-hand sides, 9 shifts, FP32 storage, blocks of 16
        dict(L=6, idx=[5, 100], M=9, opts=dict(tol=1e-9, max_iter=6000, precision="fp32", block=16)),
    ]
    order = cases if first else cases[::-1]
    for c in order:
        L = c["L"]
        Hc = simple_cubic(L, rng.uniform(-1, 1, L ** 3))
        H = S.Hamiltonian.from_csr(Hc)
        z = np.linspace(-6.5, 6.5, c["M"]) + 1j * rng.uniform(0.03, 0.3, c["M"])
        Gref, repref, _, rcref = S.greens_diag(H, z, c["idx"], **c["opts"])
        rc, G, rep = _noalloc(lib, C, H, z, c["idx"], S.options(**c["opts"]))
        assert rc == rcref == 0, lib.scocg_last_error()
        assert np.array_equal(G, Gref.cpu().numpy()), L
        assert np.array_equal(rep["iters"], repref["iters"])
        assert np.array_equal(rep["status"], repref["status"])
        assert np.array_equal(rep["rel_res_recursive"], repref["res"])
        assert S.last_timing()["switches"] >= 0


def test_noalloc_refuses_oversized_and_unsupported_requests():
    import paper_0802_0748_amd as S
    from paper_0802_0748_amd import _capi as C

    lib = C.load()
    L = 32
    Hc = simple_cubic(L, np.zeros(L ** 3))
    H = S.Hamiltonian.from_csr(Hc)
    z = np.linspace(-6, 6, 64) + 0.05j
    # 64 shifts x 8 right-hand sides x 32768 rows of FP64 directions alone are 268 MB
    rc, _, _ = _noalloc(lib, C, H, z, np.arange(8), S.options(tol=1e-8))
    assert rc == C.EINVAL and "scratch" in lib.scocg_last_error().decode()
    rc, _, _ = _noalloc(lib, C, H, z[:4], [0], S.options(tol=1e-8, window=2))
    assert rc == C.EINVAL
    rc, _, _ = _noalloc(lib, C, H, z[:4], [0], S.options(tol=1e-8, keep_tape=True))
    assert rc == C.EINVAL
