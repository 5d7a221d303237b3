"""Count sketch Kaczmarz (CSK) on AMD MI355X.

The public functions (csk_hash, csk_sketch, csk_sketch_csr, csk_solve,
csk_solve_batched, csk_solve_mrhs, ...) live in :mod:`.binding`, a thin
ctypes layer over the HIP library libcsk.so; they are loaded on first use so
that :mod:`.workloads` (seeded inputs) can be imported without the library.
Using any of them without a built libcsk.so raises ImportError.
"""
import importlib

_BINDING_NAMES = {
    "CskError", "SketchOut", "CsrSketchOut", "SolveResult", "csk_hash", "csk_sketch", "csk_sketch_csr",
    "csk_sketch_csr_sparse", "csk_solve", "csk_solve_noalloc", "csk_solve_csr_refresh", "csk_solve_csr", "csk_solve_rgrk", "csk_solve_rk",
    "csk_pipeline_capture", "Pipeline",
    "csk_solve_batched", "csk_solve_batched_sketches", "csk_solve_mrhs", "csk_tune_solve", "csk_tune_lookup", "csk_tune_clear",
    "csk_tune_mrhs", "csk_tune_batched", "csk_tune_save", "csk_tune_load",
    "csk_status_string", "parse_results", "lib",
    "CSK_OK", "CSK_NOT_CONVERGED", "CSK_ERR_INVALID_ARG", "CSK_ERR_UNSUPPORTED", "CSK_ERR_DEVICE",
    "CSK_ERR_WORKSPACE", "CSK_ERR_NONFINITE", "CSK_ERR_DEGENERATE", "CSK_CANCELLED",
    "CSK_F64", "CSK_F32", "CSK_F16", "CSK_BF16", "CSK_STOP_REL_ERR", "CSK_STOP_REL_RESID",
}


def __getattr__(name):
    if name in _BINDING_NAMES:
        return getattr(importlib.import_module(".binding", __name__), name)
    raise AttributeError(name)
