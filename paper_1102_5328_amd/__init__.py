"""MI355X-native tile Householder QR (FP64) with an empirical (NB, IB)
autotuner and a learned cost model.

The compute path is libtileqr.so (HIP kernels for gfx950 behind a C ABI,
include/tileqr.h); this package marshals torch tensors into it. PyTorch only
provides device memory and streams.

Matrices are column-major: an M x N matrix is a torch tensor with
stride(0) == 1 and stride(1) == lda >= M, e.g. ``colmajor(M, N)``.
"""
import ctypes

from . import _lib
from ._lib import TileQRError, check

__all__ = [
    "colmajor", "T_size", "factor", "apply_Qt", "factor_batched", "factor_loop", "set_compute_units", "sync",
    "tile_task", "ssrfb_bench", "ssrfb_bench_flush", "tune", "tune_units", "tune_load", "flops", "flops_executed", "dag_counts",
    "plan_check", "plan_tasks", "TileQRError", "check",
]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ld(t):
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("expected a column-major 2-D tensor (stride(0) == 1)")
    return max(1, t.stride(1)) if t.shape[1] > 1 else max(1, t.shape[0])


def colmajor(M, N, dtype=None, device="cuda", fill=None):
    """An M x N column-major tensor (lda = M)."""
    torch = _torch()
    dtype = dtype or torch.float64
    t = torch.empty((N, max(M, 1)), dtype=dtype, device=device).t()[:M]
    if fill is not None:
        t.fill_(fill)
    return t


def T_size(M, N, nb, ib, p=1):
    """Doubles of the T buffer (qr_T_size_ca; p = 1: the flat tree's)."""
    n = _lib.lib().qr_T_size_ca(M, N, nb, ib, p)
    if n < 0:
        raise TileQRError("qr_T_size_ca: invalid argument %d" % -n)
    return n


import os as _os

SHIPPED_TABLE = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "tuning",
                              "decision_table.txt")
_table_loaded = False


def _ensure_table():
    """Loads the shipped decision table once, unless the caller loaded one."""
    global _table_loaded
    if not _table_loaded:
        _table_loaded = True
        if _os.path.exists(SHIPPED_TABLE):
            check(_lib.lib().qr_tune_load(SHIPPED_TABLE.encode()), "qr_tune_load")


def tune(M, N, batch=1):
    """(NB, IB, source) from qr_tune; the shipped decision table is loaded
    on first use unless tune_load was called before."""
    _ensure_table()
    nb, ib, src = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(_lib.lib().qr_tune(M, N, batch, ctypes.byref(nb), ctypes.byref(ib), ctypes.byref(src)), "qr_tune")
    return nb.value, ib.value, src.value


def tune_units(M, N, batch=1):
    """Compute units the grid of an M x N factorization is sized for (0: all)."""
    _ensure_table()
    cus = ctypes.c_int()
    check(_lib.lib().qr_tune_units(M, N, batch, ctypes.byref(cus)), "qr_tune_units")
    return cus.value


def tune_domains(M, N, batch=1):
    """Row domains of qr_factor_ca for an M x N factorization (table; 1 when
    absent)."""
    _ensure_table()
    p = ctypes.c_int()
    check(_lib.lib().qr_tune_domains(M, N, batch, ctypes.byref(p)), "qr_tune_domains")
    return p.value


def tune_load(path):
    global _table_loaded
    check(_lib.lib().qr_tune_load(path.encode()), "qr_tune_load")
    _table_loaded = True


def factor(A, nb=0, ib=0, T=None, stream=None):
    """In-place tile QR of the column-major FP64 tensor A. Returns (A, T, nb, ib)."""
    torch = _torch()
    M, N = A.shape
    # The grid size of the launch comes from the decision table's units
    # unless set_compute_units was called: load it first, so a call sizes its
    # grid the same way whatever ran before it.
    _ensure_table()
    if nb == 0 or ib == 0:
        tnb, tib, _ = tune(M, N, 1)
        nb = nb or tnb
        ib = ib or min(tib, nb)
    if T is None:
        T = torch.empty(max(1, T_size(M, N, nb, ib)), dtype=torch.float64, device=A.device)
    check(_lib.lib().qr_factor(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib,
                               ctypes.c_void_p(T.data_ptr()), _stream(stream)), "qr_factor")
    return A, T, nb, ib


def factor_ca(A, nb, ib, p, T=None, stream=None):
    """qr_factor_ca: tile QR with p row domains merged over a binary tree
    (p = 1: the flat tree). Returns (A, T)."""
    torch = _torch()
    M, N = A.shape
    _ensure_table()
    if T is None:
        T = torch.empty(max(1, T_size(M, N, nb, ib, p)), dtype=torch.float64, device=A.device)
    check(_lib.lib().qr_factor_ca(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib, p,
                                  ctypes.c_void_p(T.data_ptr()), _stream(stream)), "qr_factor_ca")
    return A, T


def apply_Qt_ca(A, T, nb, ib, p, B, stream=None):
    """B <- Q^T B in place with Q from factor_ca (same nb, ib, p)."""
    M, N = A.shape
    _ensure_table()
    check(_lib.lib().qr_apply_Qt_ca(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib, p,
                                    ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                    B.shape[1], _ld(B), _stream(stream)), "qr_apply_Qt_ca")
    return B


def apply_Q(A, T, nb, ib, B, p=1, stream=None):
    """B <- Q B in place (qr_apply_Q_ca; same nb, ib, p as the factorization)."""
    M, N = A.shape
    _ensure_table()
    check(_lib.lib().qr_apply_Q_ca(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib, p,
                                   ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                   B.shape[1], _ld(B), _stream(stream)), "qr_apply_Q_ca")
    return B


def form_Q(A, T, nb, ib, k=None, p=1, Q=None, stream=None):
    """The first k columns of Q (default min(M, N)) as an M x k column-major
    tensor (qr_form_Q_ca)."""
    M, N = A.shape
    k = min(M, N) if k is None else k
    if Q is None:
        Q = colmajor(M, k, device=A.device)
    _ensure_table()
    check(_lib.lib().qr_form_Q_ca(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib, p,
                                  ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(Q.data_ptr()),
                                  k, _ld(Q), _stream(stream)), "qr_form_Q_ca")
    return Q


def solve_ls(A, T, nb, ib, B, p=1, stream=None):
    """Least squares for M >= N in place: B <- [X; Q^T residual] with X in
    the first N rows (qr_solve_ls_ca)."""
    M, N = A.shape
    _ensure_table()
    check(_lib.lib().qr_solve_ls_ca(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib, p,
                                    ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                    B.shape[1], _ld(B), _stream(stream)), "qr_solve_ls_ca")
    return B


def factor_noalloc(A, nb, ib, T, stream=None):
    """qr_factor_noalloc: the factorization without device allocations (T
    supplied by the caller; the library's static scratch holds the rest)."""
    M, N = A.shape
    check(_lib.lib().qr_factor_noalloc(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib,
                                       ctypes.c_void_p(T.data_ptr()), _stream(stream)),
          "qr_factor_noalloc")
    return A, T


def apply_Qt(A, T, nb, ib, B, stream=None):
    """B <- Q^T B in place (B column-major, M rows)."""
    M, N = A.shape
    _ensure_table()
    check(_lib.lib().qr_apply_Qt(ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib,
                                 ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                 B.shape[1], _ld(B), _stream(stream)), "qr_apply_Qt")
    return B


def _batch_args(As, nbs, ibs, Ts):
    n = len(As)
    P = ctypes.c_void_p * n
    I64 = ctypes.c_int64 * n
    INT = ctypes.c_int * n
    a = P(*[ctypes.c_void_p(x.data_ptr()) for x in As])
    m = I64(*[x.shape[0] for x in As])
    nn = I64(*[x.shape[1] for x in As])
    ld = I64(*[_ld(x) for x in As])
    t = P(*[ctypes.c_void_p(x.data_ptr()) for x in Ts])
    return a, m, nn, ld, INT(*nbs), INT(*ibs), t


def factor_batched(As, nbs, ibs, Ts, stream=None):
    """One persistent, graph-captured launch over all matrices."""
    _ensure_table()
    a, m, n, ld, nb, ib, t = _batch_args(As, nbs, ibs, Ts)
    check(_lib.lib().qr_factor_batched(ctypes.cast(a, ctypes.c_void_p), m, n, ld, len(As), nb, ib,
                                       ctypes.cast(t, ctypes.c_void_p), _stream(stream)),
          "qr_factor_batched")


def factor_loop(As, nbs, ibs, Ts, stream=None):
    """One qr_factor launch per matrix (the baseline of the batched launch)."""
    _ensure_table()
    a, m, n, ld, nb, ib, t = _batch_args(As, nbs, ibs, Ts)
    check(_lib.lib().qr_factor_loop(ctypes.cast(a, ctypes.c_void_p), m, n, ld, len(As), nb, ib,
                                    ctypes.cast(t, ctypes.c_void_p), _stream(stream)),
          "qr_factor_loop")


def set_compute_units(cus):
    """Grid and schedule for `cus` compute units (0: all); see the header."""
    check(_lib.lib().qr_set_compute_units(cus), "qr_set_compute_units")


def sync(stream=None):
    check(_lib.lib().qr_sync(_stream(stream)), "qr_sync")


def trace_fetch():
    """Per-task trace of the last factorization run with TILEQR_TRACE=1:
    an (ntasks, 9) int64 array (type, i, j, k, strip, t_take, t_ready,
    t_done in ns, workgroup)."""
    import numpy as np
    n = ctypes.c_int64()
    check(_lib.lib().qr_trace_fetch(None, 0, ctypes.byref(n)), "qr_trace_fetch")
    out = np.zeros((max(1, n.value), 9), dtype=np.int64)
    check(_lib.lib().qr_trace_fetch(out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n.value,
                                    ctypes.byref(n)), "qr_trace_fetch")
    return out[:n.value]


def tile_task(kind, A, nb, ib, T, i, j, k, stream=None):
    M, N = A.shape
    check(_lib.lib().qr_tile_task(kind, ctypes.c_void_p(A.data_ptr()), M, N, _ld(A), nb, ib,
                                  ctypes.c_void_p(T.data_ptr()), i, j, k, _stream(stream)),
          "qr_tile_task")


def ssrfb_bench(nb, ib, calls=50, workers=0):
    sec = ctypes.c_double()
    check(_lib.lib().qr_ssrfb_bench(nb, ib, calls, workers, ctypes.byref(sec)), "qr_ssrfb_bench")
    return sec.value


def ssrfb_bench_flush(nb, ib, calls=50, workers=0, flush_bytes=1 << 30):
    sec = ctypes.c_double()
    check(_lib.lib().qr_ssrfb_bench_flush(nb, ib, calls, workers, flush_bytes, ctypes.byref(sec)),
          "qr_ssrfb_bench_flush")
    return sec.value


def mfma_probe(wg_per_cu=2, iters=50000):
    """qr_mfma_probe: the sustained FP64 MFMA rate of the chip (TFLOP/s) and
    the shader clock (GHz) measured over the probe's run."""
    tf, ghz = ctypes.c_double(), ctypes.c_double()
    check(_lib.lib().qr_mfma_probe(wg_per_cu, iters, ctypes.byref(tf), ctypes.byref(ghz)),
          "qr_mfma_probe")
    return tf.value, ghz.value


def flops(M, N):
    return _lib.lib().qr_flops(M, N)


def flops_executed(M, N, nb, ib):
    return _lib.lib().qr_flops_executed(M, N, nb, ib)


def dag_counts(M, N, nb):
    c = (ctypes.c_int64 * 4)()
    check(_lib.lib().qr_dag_counts(M, N, nb, c), "qr_dag_counts")
    return list(c)


def plan_check(M, N, nb, ib, nrhs=0, apply=False, workers=256, seed=0, p=1):
    nt, seq, stress = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(_lib.lib().qr_plan_check(M, N, nb, ib, p, nrhs, int(apply), workers, seed, ctypes.byref(nt),
                                   ctypes.byref(seq), ctypes.byref(stress)), "qr_plan_check")
    return nt.value, seq.value, stress.value


def plan_tasks(M, N, nb, ib, nrhs=0, apply=False, workers=256, p=1):
    import numpy as np
    nt = ctypes.c_int64()
    check(_lib.lib().qr_plan_tasks(M, N, nb, ib, p, nrhs, int(apply), workers, None, 0,
                                   ctypes.byref(nt)), "qr_plan_tasks")
    out = np.zeros((max(1, nt.value), 5), dtype=np.int32)
    check(_lib.lib().qr_plan_tasks(M, N, nb, ib, p, nrhs, int(apply), workers,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nt.value,
                                   ctypes.byref(nt)), "qr_plan_tasks")
    return out[:nt.value]
