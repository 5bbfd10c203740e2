"""CPU checks of the C ABI: the library loads, exports every declared entry point,
and its host-only helpers (matrix validation, contour nodes) behave as documented."""

import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "scocg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", src, flags=re.M)) - {"if", "extern"})


def test_library_exports_every_declared_function():
    from paper_0802_0748_amd import _capi as C

    lib = C.load()
    names = _declared()
    assert "shifted_cocg_solve" in names and "backward" in names and "csr_upload" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(C.EXPORTED) <= set(names)


def test_opts_struct_layout():
    import ctypes

    from paper_0802_0748_amd import _capi as C

    o = C.Opts()
    C.load().scocg_default_opts(ctypes.byref(o))
    assert o.tol == 1e-8 and o.max_iter == 3000 and o.seed_index == -1 and o.seed_switching == 1
    assert ctypes.sizeof(C.Opts) == 8 + 4 * 15 + 4  # padded to 8 bytes
    assert C.Opts.window.offset == 8 + 4 * 11 and C.Opts.schedule.offset == 8 + 4 * 12
    assert ctypes.sizeof(C.PairReport) == 24
    # the timing record: fields appended at the end keep the offsets of the earlier ones
    assert ctypes.sizeof(C.Timing) == 64 and C.Timing.update_flops.offset == 56
    t = C.Timing()
    assert C.load().scocg_last_timing(ctypes.byref(t)) == 0 and t.update_flops >= 0.0


def test_validation_rejects_bad_matrices():
    from paper_0802_0748_amd import _capi as C
    from paper_0802_0748_amd.api import csr_validate
    from workloads import random_sparse_symmetric

    H = random_sparse_symmetric(12, 0.3, np.random.default_rng(0))
    csr_validate(H.row_ptr, H.col, H.val)
    bad_val = H.val.copy()
    off = np.nonzero(np.repeat(np.arange(12), np.diff(H.row_ptr)) != H.col)[0][0]
    bad_val[off] += 1e-12
    with pytest.raises(C.ScocgError):
        csr_validate(H.row_ptr, H.col, bad_val)
    nan_val = H.val.copy()
    nan_val[0] = np.inf
    with pytest.raises(C.ScocgError):
        csr_validate(H.row_ptr, H.col, nan_val)
    unsorted = H.col.copy()
    r0 = slice(H.row_ptr[0], H.row_ptr[1])
    if H.row_ptr[1] - H.row_ptr[0] >= 2:
        unsorted[r0] = unsorted[r0][::-1]
        with pytest.raises(C.ScocgError):
            csr_validate(H.row_ptr, unsorted, H.val)
    oob = H.col.copy()
    oob[-1] = 12
    with pytest.raises(C.ScocgError):
        csr_validate(H.row_ptr, oob, H.val)
    asym_rp = np.array([0, 1, 1], dtype=np.int64)
    with pytest.raises(C.ScocgError):
        csr_validate(asym_rp, np.array([1]), np.array([1.0]))


def test_contour_nodes_match_oracle_quadrature():
    """The library's Gauss-Legendre contour equals the oracle's (numpy leggauss) nodes."""
    from oracle import oracle as O
    from paper_0802_0748_amd.api import contour

    for nq in (1, 7, 128):
        z, w = contour(-13.0, 0.0, nq)
        z2, w2 = O.contour(-13.0, 0.0, nq)
        assert np.max(np.abs(z - z2)) < 1e-12
        assert np.max(np.abs(w - w2)) < 1e-12


def test_bindings_refuse_host_buffers():
    """Every pointer the bindings hand to the library must be device memory: host tensors and
    host output devices are refused before any call (no GPU needed for the checks)."""
    import torch

    from paper_0802_0748_amd import api

    with pytest.raises(ValueError):
        api._device("cpu")
    assert api._device(None).type == "cuda"
    with pytest.raises(ValueError):
        api._check_dev(torch.zeros(4, dtype=torch.complex128), torch.complex128, 4, "out")


def test_null_arguments_are_refused_without_a_device():
    """Null handles or buffers are EINVAL with a message, decided before any device work
    (so this runs on the CPU)."""
    import ctypes

    from paper_0802_0748_amd import _capi as C

    lib = C.load()
    o = C.Opts()
    lib.scocg_default_opts(ctypes.byref(o))
    z = np.array([0.0, 0.1])
    assert lib.greens_proj(None, 1, z.ctypes.data, 1, None, None, ctypes.byref(o), None, None, None) == C.EINVAL
    assert "null" in lib.scocg_last_error().decode()
    assert lib.shifted_cocg_solve(None, 1, z.ctypes.data, 1, None, ctypes.byref(o), None, None, None, None) == C.EINVAL
    assert lib.krylov_greens_diag(None, 1, z.ctypes.data, 1, None, 4, None, None, None, None) == C.EINVAL
    assert lib.hubbard_fermion_op(6, 3, 3, 0, 0, 0, None, None, None) == C.EINVAL


def test_product_path_fails_loudly(monkeypatch, tmp_path):
    """There is no CPU fallback: without a HIP device every entry of the binding raises, and a
    missing library is an ImportError, never a silent substitute."""
    import torch

    from paper_0802_0748_amd import _capi as C
    from paper_0802_0748_amd import api
    from workloads import random_sparse_symmetric

    if not torch.cuda.is_available():
        H = random_sparse_symmetric(12, 0.3, np.random.default_rng(0))
        with pytest.raises(RuntimeError, match="HIP device"):
            api.Hamiltonian.from_csr(H)
        with pytest.raises(RuntimeError, match="HIP device"):
            api.Hamiltonian.hubbard(6, 3, 3)
        with pytest.raises(RuntimeError, match="HIP device"):
            api.greens_diag(None, [0.1j], [0])
    monkeypatch.setattr(C, "_lib", None)
    monkeypatch.setattr(C, "LIB_PATH", str(tmp_path / "libscocg.so"))
    with pytest.raises(ImportError, match="not built"):
        C.load()
