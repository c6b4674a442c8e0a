"""ctypes binding of libtileqr.so: the same names as include/tileqr.h.

Argument marshalling only: every step of the path runs in the library's
HIP kernels. Loading fails loudly if the library has not been built; there
is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtileqr.so")

_lib = None

c_i64 = ctypes.c_int64
c_int = ctypes.c_int
c_u64 = ctypes.c_uint64
c_dbl = ctypes.c_double
c_flt = ctypes.c_float
c_vp = ctypes.c_void_p
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_intp = ctypes.POINTER(ctypes.c_int)
c_i32p = ctypes.POINTER(ctypes.c_int32)
c_dblp = ctypes.POINTER(ctypes.c_double)
c_fltp = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes)
SIGNATURES = {
    "qr_version": (ctypes.c_char_p, []),
    "qr_T_size": (c_i64, [c_i64, c_i64, c_int, c_int]),
    "qr_T_size_ca": (c_i64, [c_i64, c_i64, c_int, c_int, c_int]),
    "qr_factor_ca": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_int, c_vp, c_vp]),
    "qr_apply_Qt_ca": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_int, c_vp, c_vp, c_i64, c_i64, c_vp]),
    "qr_apply_Q_ca": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_int, c_vp, c_vp, c_i64, c_i64, c_vp]),
    "qr_apply_Q": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_vp, c_vp, c_i64, c_i64, c_vp]),
    "qr_form_Q_ca": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_int, c_vp, c_vp, c_i64, c_i64, c_vp]),
    "qr_solve_ls_ca": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_int, c_vp, c_vp, c_i64, c_i64, c_vp]),
    "qr_factor": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_vp, c_vp]),
    "qr_factor_noalloc": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_vp, c_vp]),
    "qr_apply_Qt": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_vp, c_vp, c_i64, c_i64, c_vp]),
    "qr_factor_batched": (c_int, [c_vp, c_i64p, c_i64p, c_i64p, c_i64, c_intp, c_intp, c_vp, c_vp]),
    "qr_factor_loop": (c_int, [c_vp, c_i64p, c_i64p, c_i64p, c_i64, c_intp, c_intp, c_vp, c_vp]),
    "qr_sync": (c_int, [c_vp]),
    "qr_set_compute_units": (c_int, [c_int]),
    "qr_trace_fetch": (c_int, [c_i64p, c_i64, c_i64p]),
    "qr_tile_task": (c_int, [c_int, c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_vp, c_int, c_int, c_int, c_vp]),
    "qr_ssrfb_bench": (c_int, [c_int, c_int, c_int, c_int, c_dblp]),
    "qr_ssrfb_bench_flush": (c_int, [c_int, c_int, c_int, c_int, c_i64, c_dblp]),
    "qr_mfma_probe": (c_int, [c_int, c_int, c_dblp, c_dblp]),
    "qr_tune": (c_int, [c_i64, c_i64, c_i64, c_intp, c_intp, c_intp]),
    "qr_tune_load": (c_int, [ctypes.c_char_p]),
    "qr_tune_units": (c_int, [c_i64, c_i64, c_i64, c_intp]),
    "qr_tune_domains": (c_int, [c_i64, c_i64, c_i64, c_intp]),
    "qr_tune_set_model": (c_int, [c_fltp, c_int, c_fltp, c_fltp, c_flt, c_flt, c_intp, c_int]),
    "qr_mlp_forward": (c_int, [c_vp, c_int, c_vp, c_i64, c_vp, c_vp]),
    "qr_mlp_grad": (c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "qr_mlp_train": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_i64, c_int, c_int, c_flt, c_u64, c_i64, c_vp, c_vp]),
    "qr_dag_counts": (c_int, [c_i64, c_i64, c_int, c_i64p]),
    "qr_flops": (c_dbl, [c_i64, c_i64]),
    "qr_flops_executed": (c_dbl, [c_i64, c_i64, c_int, c_int]),
    "qr_plan_check": (c_int, [c_i64, c_i64, c_int, c_int, c_int, c_i64, c_int, c_int, c_u64, c_i64p, c_i64p, c_i64p]),
    "qr_plan_tasks": (c_int, [c_i64, c_i64, c_int, c_int, c_int, c_i64, c_int, c_int, c_i32p, c_i64, c_i64p]),
}


class TileQRError(RuntimeError):
    pass


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TileQRError(
                "libtileqr.so not built: run `python -m paper_1102_5328_amd.build` "
                "(or __graft_entry__.build())")
        # torch ships its own HIP runtime; load it first so that the library
        # binds to the same one (one runtime per process, one device context).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc, what):
    if rc != 0:
        raise TileQRError("%s failed with code %d" % (what, rc))
    return rc


def __getattr__(name):  # module-level passthrough: _lib.qr_factor(...)
    if name in SIGNATURES:
        return getattr(lib(), name)
    raise AttributeError(name)
