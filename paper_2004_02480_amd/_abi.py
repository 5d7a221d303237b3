"""ctypes declarations of libcsk's C ABI (include/csk.h).

Argument marshalling only: every computation happens in the HIP library.  If
the library has not been built this module raises at import time; there is no
fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsk.so")

# status codes
CSK_OK = 0
CSK_NOT_CONVERGED = 1
CSK_ERR_INVALID_ARG = 2
CSK_ERR_UNSUPPORTED = 3
CSK_ERR_DEVICE = 4
CSK_ERR_WORKSPACE = 5
CSK_ERR_NONFINITE = 6
CSK_ERR_DEGENERATE = 7
CSK_CANCELLED = 8

# dtypes
CSK_F64 = 0
CSK_F32 = 1
CSK_F16 = 2
CSK_BF16 = 3

CSK_STOP_REL_ERR = 0
CSK_STOP_REL_RESID = 1

EXPORTED = [
    "csk_status_string", "csk_last_error", "csk_version", "csk_hash",
    "csk_sketch_workspace_size", "csk_sketch",
    "csk_sketch_csr_workspace_size", "csk_sketch_csr",
    "csk_sketch_csr_sparse_workspace_size", "csk_sketch_csr_sparse",
    "csk_solve_workspace_size", "csk_solve", "csk_solve_noalloc",
    "csk_solve_csr_refresh_workspace_size", "csk_solve_csr_refresh",
    "csk_solve_csr_workspace_size", "csk_solve_csr",
    "csk_solve_rgrk_workspace_size", "csk_solve_rgrk",
    "csk_solve_rk_workspace_size", "csk_solve_rk",
    "csk_pipeline_capture", "csk_pipeline_launch", "csk_pipeline_destroy",
    "csk_solve_batched_workspace_size", "csk_solve_batched", "csk_solve_batched_sketch_loc",
    "csk_solve_mrhs_workspace_size", "csk_solve_mrhs",
    "csk_tune_solve_workspace_size", "csk_tune_solve", "csk_tune_lookup", "csk_tune_clear",
    "csk_tune_mrhs_workspace_size", "csk_tune_mrhs", "csk_tune_batched", "csk_tune_save", "csk_tune_load",
]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int64),
        ("stop_mode", ctypes.c_int32),
        ("refresh_every", ctypes.c_int32),
        ("x_ref", ctypes.c_void_p),
        ("cancel", ctypes.c_void_p),
        ("check_every", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("single_wg", ctypes.c_int32),
        ("trace_idx", ctypes.c_void_p),
    ]


class SystemDesc(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p),
        ("b", ctypes.c_void_p),
        ("x_ref", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("d", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
    ]


class BatchedSketchLoc(ctypes.Structure):
    _fields_ = [
        ("at64", ctypes.c_int64),
        ("at_lp", ctypes.c_int64),
        ("bt", ctypes.c_int64),
        ("nu2", ctypes.c_int64),
        ("ld64", ctypes.c_int64),
        ("ld_lp", ctypes.c_int64),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_int32),
        ("lanes_per_row", ctypes.c_int32),
        ("us_per_iter", ctypes.c_double),
    ]


class TuneReport(ctypes.Structure):
    _fields_ = [
        ("choice", ctypes.c_int32),
        ("default_choice", ctypes.c_int32),
        ("us", ctypes.c_double),
        ("default_us", ctypes.c_double),
        ("candidates", ctypes.c_int32),
    ]


# the static scratch of csk_solve_noalloc (CSK_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 8 << 20

# csk_solve_result: int64 iters; int32 status; int32 fp64_fallback;
# double final_measure; int64 refreshes  -> 32 bytes
RESULT_BYTES = 32


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"libcsk.so not found at {path}; build it first with "
            "`python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_2004_02480_amd/build.py`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I32 = ctypes.c_int32
    U64 = ctypes.c_uint64
    SZ = ctypes.c_size_t
    PSZ = ctypes.POINTER(ctypes.c_size_t)
    lib.csk_status_string.restype = ctypes.c_char_p
    lib.csk_status_string.argtypes = [I32]
    lib.csk_last_error.restype = ctypes.c_char_p
    lib.csk_last_error.argtypes = []
    lib.csk_version.restype = I32
    lib.csk_version.argtypes = []
    lib.csk_hash.restype = I32
    lib.csk_hash.argtypes = [U64, I64, I64, P, P, P]
    lib.csk_sketch_workspace_size.restype = I32
    lib.csk_sketch_workspace_size.argtypes = [I64, I64, I64, I64, PSZ]
    lib.csk_sketch.restype = I32
    lib.csk_sketch.argtypes = [P, I32, I64, I64, I64, P, I64, I64, I64, U64,
                               P, I64, P, I32, I64, P, I64, P, P, P, P, SZ, P]
    lib.csk_sketch_csr_workspace_size.restype = I32
    lib.csk_sketch_csr_workspace_size.argtypes = [I64, I64, I64, PSZ]
    lib.csk_sketch_csr.restype = I32
    lib.csk_sketch_csr.argtypes = [P, P, P, I64, I64, I64, P, I64, U64,
                                   P, I64, P, I32, I64, P, P, P, SZ, P]
    lib.csk_sketch_csr_sparse_workspace_size.restype = I32
    lib.csk_sketch_csr_sparse_workspace_size.argtypes = [I64, I64, I64, PSZ]
    lib.csk_sketch_csr_sparse.restype = I32
    lib.csk_sketch_csr_sparse.argtypes = [P, P, P, I64, I64, I64, P, I64, U64,
                                          P, P, P, P, P, P, SZ, P]
    lib.csk_solve_csr_workspace_size.restype = I32
    lib.csk_solve_csr_workspace_size.argtypes = [I64, I64, I64, PSZ]
    lib.csk_solve_csr.restype = I32
    lib.csk_solve_csr.argtypes = [P, P, P, I64, I64, I64, P, P, P, P,
                                  ctypes.POINTER(SolveOpts), P, P, SZ, P]
    lib.csk_solve_rgrk_workspace_size.restype = I32
    lib.csk_solve_rgrk_workspace_size.argtypes = [I64, I64, PSZ]
    lib.csk_solve_rgrk.restype = I32
    lib.csk_solve_rgrk.argtypes = [P, I64, I64, I64, P, P, P, P, ctypes.c_double, U64,
                                   ctypes.POINTER(SolveOpts), P, P, SZ, P]
    lib.csk_solve_rk_workspace_size.restype = I32
    lib.csk_solve_rk_workspace_size.argtypes = [I64, I64, PSZ]
    lib.csk_solve_rk.restype = I32
    lib.csk_solve_rk.argtypes = [P, I64, I64, I64, P, P, P, P, U64,
                                 ctypes.POINTER(SolveOpts), P, P, SZ, P]
    lib.csk_pipeline_capture.restype = I32
    lib.csk_pipeline_capture.argtypes = [P, I32, I64, I64, I64, P, I64, U64, P, I64, P, I32, I64, P, P, P, P,
                                         ctypes.POINTER(SolveOpts), P, P, SZ, P, SZ, P,
                                         ctypes.POINTER(ctypes.c_void_p)]
    lib.csk_pipeline_launch.restype = I32
    lib.csk_pipeline_launch.argtypes = [P, P]
    lib.csk_pipeline_destroy.restype = I32
    lib.csk_pipeline_destroy.argtypes = [P]
    lib.csk_solve_workspace_size.restype = I32
    lib.csk_solve_workspace_size.argtypes = [I64, I64, I32, PSZ]
    lib.csk_solve.restype = I32
    lib.csk_solve.argtypes = [P, I32, I64, P, I64, I64, I64, P, P, P, P,
                              ctypes.POINTER(SolveOpts), P, P, SZ, P]
    lib.csk_solve_csr_refresh_workspace_size.restype = I32
    lib.csk_solve_csr_refresh_workspace_size.argtypes = [I64, I64, I64, PSZ]
    lib.csk_solve_csr_refresh.restype = I32
    lib.csk_solve_csr_refresh.argtypes = [P, I32, I64, P, I64, I64, I64, P, P, P, I64, P, U64, P, P, P, P,
                                          ctypes.POINTER(SolveOpts), P, P, SZ, P]
    lib.csk_solve_noalloc.restype = I32
    lib.csk_solve_noalloc.argtypes = [P, I32, I64, P, I64, I64, I64, P, P, P, P,
                                      ctypes.POINTER(SolveOpts), P, P]
    lib.csk_solve_batched_workspace_size.restype = I32
    lib.csk_solve_batched_workspace_size.argtypes = [ctypes.POINTER(SystemDesc), I32, I32, I32, PSZ]
    lib.csk_solve_batched_sketch_loc.restype = I32
    lib.csk_solve_batched_sketch_loc.argtypes = [ctypes.POINTER(SystemDesc), I32, I32, I32, I32,
                                                 ctypes.POINTER(BatchedSketchLoc)]
    lib.csk_solve_batched.restype = I32
    lib.csk_solve_batched.argtypes = [ctypes.POINTER(SystemDesc), I32, I32, I32,
                                      ctypes.POINTER(SolveOpts), P, P, SZ, P]
    lib.csk_solve_mrhs_workspace_size.restype = I32
    lib.csk_solve_mrhs_workspace_size.argtypes = [I64, I64, I64, PSZ]
    lib.csk_solve_mrhs.restype = I32
    lib.csk_solve_mrhs.argtypes = [P, I32, I64, P, I64, I64, I64, P, I64, I64, P,
                                   P, P, I64, P, I64, ctypes.POINTER(SolveOpts), P, P, SZ, P]
    lib.csk_tune_solve_workspace_size.restype = I32
    lib.csk_tune_solve_workspace_size.argtypes = [I64, I64, I32, PSZ]
    lib.csk_tune_solve.restype = I32
    lib.csk_tune_solve.argtypes = [P, I32, I64, P, I64, I64, I64, P, P, I32, ctypes.POINTER(TuneEntry), P, SZ, P]
    lib.csk_tune_lookup.restype = I32
    lib.csk_tune_lookup.argtypes = [I64, I64, I32, I32, ctypes.POINTER(TuneEntry)]
    lib.csk_tune_clear.restype = None
    lib.csk_tune_clear.argtypes = []
    lib.csk_tune_mrhs_workspace_size.restype = I32
    lib.csk_tune_mrhs_workspace_size.argtypes = [I64, I64, I64, PSZ]
    lib.csk_tune_mrhs.restype = I32
    lib.csk_tune_mrhs.argtypes = [P, I32, I64, P, I64, I64, I64, P, I64, I64, P, I32, ctypes.POINTER(TuneReport),
                                  P, SZ, P]
    lib.csk_tune_batched.restype = I32
    lib.csk_tune_batched.argtypes = [ctypes.POINTER(SystemDesc), I32, I32, I32, ctypes.POINTER(SolveOpts), P,
                                     ctypes.POINTER(TuneReport), P, SZ, P]
    lib.csk_tune_save.restype = I32
    lib.csk_tune_save.argtypes = [ctypes.c_char_p]
    lib.csk_tune_load.restype = I32
    lib.csk_tune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(I32)]
    return lib
