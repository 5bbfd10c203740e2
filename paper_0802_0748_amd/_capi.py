"""ctypes declarations of libscocg.so (the C ABI in include/scocg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
If the library is missing or cannot be loaded, this module raises; there is no
fallback implementation.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscocg.so")

OK, EINVAL, ENOMEM, EHIP, EBREAKDOWN, ENOCONV = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "EBREAKDOWN", 5: "ENOCONV"}


class Opts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("seed_index", ctypes.c_int32),
        ("seed_switching", ctypes.c_int32),
        ("fixed_iter", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("shifts_per_wg", ctypes.c_int32),
        ("check_true", ctypes.c_int32),
        ("keep_tape", ctypes.c_int32),
        ("no_graph", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("window", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("update_form", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class PairReport(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("rel_res_recursive", ctypes.c_double),
        ("rel_res_true", ctypes.c_double),
    ]


class Timing(ctypes.Structure):
    _fields_ = [
        ("update_ms", ctypes.c_double),
        ("update_launches", ctypes.c_int64),
        ("update_bytes", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("iterations", ctypes.c_int64),
        ("blocks", ctypes.c_int64),
        ("switches", ctypes.c_int64),
        ("update_flops", ctypes.c_double),
    ]


EXPORTED = [
    "scocg_default_opts",
    "scocg_csr_validate",
    "csr_upload",
    "hubbard_upload",
    "csr_update_values",
    "csr_n",
    "csr_nnz",
    "csr_free",
    "shifted_cocg_solve",
    "greens_diag",
    "greens_diag_noalloc",
    "greens_diag_batched",
    "greens_proj",
    "krylov_greens_diag",
    "krylov_greens_vec",
    "ground_state",
    "hubbard_fermion_op",
    "density_matrix_energy",
    "backward",
    "tape_free",
    "scocg_contour",
    "scocg_last_error",
    "scocg_last_timing",
    "scocg_set_profiling",
    "scocg_last_switches",
]

_lib = None


def load():
    """Load libscocg.so and declare its prototypes (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_0802_0748_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int
    lib.scocg_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.scocg_default_opts.restype = None
    lib.scocg_csr_validate.argtypes = [i64, i64, P, P, P]
    lib.scocg_csr_validate.restype = i32
    lib.csr_upload.argtypes = [i64, i64, P, P, P, i32, P, ctypes.POINTER(P)]
    lib.csr_upload.restype = i32
    lib.hubbard_upload.argtypes = [i32, i32, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, P,
                                   ctypes.POINTER(P)]
    lib.hubbard_upload.restype = i32
    lib.krylov_greens_diag.argtypes = [P, i64, P, i64, P, i32, P, P, P, P]
    lib.krylov_greens_diag.restype = i32
    lib.krylov_greens_vec.argtypes = [P, i64, P, P, i32, P, P, P, P]
    lib.krylov_greens_vec.restype = i32
    lib.ground_state.argtypes = [P, P, i32, ctypes.c_double, i32, P, P, P, P, P]
    lib.ground_state.restype = i32
    lib.hubbard_fermion_op.argtypes = [i32, i32, i32, i32, i32, i32, P, P, P]
    lib.hubbard_fermion_op.restype = i32
    lib.csr_update_values.argtypes = [P, P, P]
    lib.csr_update_values.restype = i32
    lib.csr_n.argtypes = [P]
    lib.csr_n.restype = i64
    lib.csr_nnz.argtypes = [P]
    lib.csr_nnz.restype = i64
    lib.csr_free.argtypes = [P]
    lib.csr_free.restype = None
    lib.shifted_cocg_solve.argtypes = [P, i64, P, i64, P, ctypes.POINTER(Opts), P, P, ctypes.POINTER(P), P]
    lib.shifted_cocg_solve.restype = i32
    lib.greens_diag.argtypes = [P, i64, P, i64, P, ctypes.POINTER(Opts), P, P, ctypes.POINTER(P), P]
    lib.greens_diag.restype = i32
    lib.greens_diag_noalloc.argtypes = [P, i64, P, i64, P, ctypes.POINTER(Opts), P, P, P]
    lib.greens_diag_noalloc.restype = i32
    lib.greens_diag_batched.argtypes = [i64, P, P, P, i64, P, ctypes.POINTER(Opts), P, P, P]
    lib.greens_diag_batched.restype = i32
    lib.greens_proj.argtypes = [P, i64, P, i64, P, P, ctypes.POINTER(Opts), P, P, P]
    lib.greens_proj.restype = i32
    lib.density_matrix_energy.argtypes = [P, i64, P, P, i64, P, ctypes.POINTER(Opts), i64, P, P, P, P]
    lib.density_matrix_energy.restype = i32
    lib.backward.argtypes = [P, P, P, P]
    lib.backward.restype = i32
    lib.tape_free.argtypes = [P]
    lib.tape_free.restype = None
    lib.scocg_contour.argtypes = [ctypes.c_double, ctypes.c_double, i64, P, P]
    lib.scocg_contour.restype = i32
    lib.scocg_last_error.argtypes = []
    lib.scocg_last_error.restype = ctypes.c_char_p
    lib.scocg_last_timing.argtypes = [ctypes.POINTER(Timing)]
    lib.scocg_last_timing.restype = i32
    lib.scocg_set_profiling.argtypes = [i32]
    lib.scocg_set_profiling.restype = None
    lib.scocg_last_switches.argtypes = [i64, P, i32]
    lib.scocg_last_switches.restype = ctypes.c_int32
    _lib = lib
    return lib


class ScocgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int, allow=(OK,)):
    if code not in allow:
        raise ScocgError(code, load().scocg_last_error().decode())
    return code
