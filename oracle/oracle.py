"""Python face of the CPU oracle (oracle.c). TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg import this module. It shares no code with the HIP library and never
imports it. Everything is FP64, column-major (Fortran order) numpy arrays.

Functions mirror the plain definitions in oracle.c:
  geqr2(A)            -> (R/V packed as LAPACK xGEQR2 returns them, tau)
  apply_qt(V, tau, B) -> Q^T B    (reflectors one at a time, ascending)
  apply_q(V, tau, B)  -> Q B      (descending)
  form_q(V, tau, M, K)-> thin Q, M x K
  trsv_upper(R, B)    -> R^{-1} B (back substitution), lstsq(A, B) -> X, Q^T B
  larft(V, tau, j0,k) -> compact-WY T of reflectors j0..j0+k-1
  gram_entry(A, i, j) -> (A^T A)_ij
  mlp_forward / mlp_grad (FP64 chain rule for the 5-64-64-64-1 ReLU MLP)
plus small numpy helpers for the comparisons the paper's method allows
(R after row-sign normalisation, the residual and orthogonality invariants).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

EPS = np.finfo(np.float64).eps  # 2^-52


def build(force=True):
    """Compile oracle.c with gcc (no -ffast-math: IEEE semantics kept)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, dp, dbl = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_double
    lib.oracle_geqr2.argtypes = [i64, i64, dp, i64, dp]
    lib.oracle_geqr2_steps.argtypes = [i64, i64, dp, i64, dp, i64]
    lib.oracle_apply_qt.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
    lib.oracle_apply_q.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
    lib.oracle_larft.argtypes = [i64, i64, i64, dp, i64, dp, dp, i64]
    lib.oracle_trsv_upper.argtypes = [i64, dp, i64, i64, dp, i64]
    lib.oracle_gram_entry.argtypes = [i64, dp, i64, i64, i64]
    lib.oracle_gram_entry.restype = dbl
    lib.oracle_mlp_forward.argtypes = [dp, dp, i64, dp]
    lib.oracle_mlp_grad.argtypes = [dp, dp, dp, i64, dp]
    lib.oracle_mlp_grad.restype = dbl
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fortran(a):
    return np.array(a, dtype=np.float64, order="F", copy=True)


def num_threads():
    return int(_load().oracle_num_threads())


def geqr2(A):
    """Unblocked Householder QR of a copy of A. Returns (VR, tau): R in the
    upper triangle/trapezoid, reflector tails below the diagonal."""
    a = _fortran(A)
    m, n = a.shape
    tau = np.zeros(max(1, min(m, n)), dtype=np.float64)
    _load().oracle_geqr2(m, n, _p(a), max(1, m), _p(tau))
    return a, tau[:min(m, n)]


def geqr2_steps_inplace(a, steps):
    """First `steps` Householder steps, in place on a Fortran-ordered array
    (the bounded sample the benchmark times). Returns tau."""
    assert a.flags.f_contiguous and a.dtype == np.float64
    m, n = a.shape
    tau = np.zeros(max(1, min(m, n, steps)), dtype=np.float64)
    _load().oracle_geqr2_steps(m, n, _p(a), max(1, m), _p(tau), steps)
    return tau


def apply_qt(VR, tau, B):
    """Q^T B with Q = H_0 ... H_{K-1} stored in VR/tau."""
    v = np.asfortranarray(VR, dtype=np.float64)
    b = _fortran(B if B.ndim == 2 else B.reshape(-1, 1))
    m = v.shape[0]
    t = np.ascontiguousarray(tau, dtype=np.float64)
    _load().oracle_apply_qt(m, len(t), _p(v), max(1, m), _p(t), b.shape[1], _p(b), max(1, m))
    return b


def apply_q(VR, tau, B):
    """Q B."""
    v = np.asfortranarray(VR, dtype=np.float64)
    b = _fortran(B if B.ndim == 2 else B.reshape(-1, 1))
    m = v.shape[0]
    t = np.ascontiguousarray(tau, dtype=np.float64)
    _load().oracle_apply_q(m, len(t), _p(v), max(1, m), _p(t), b.shape[1], _p(b), max(1, m))
    return b


def form_q(VR, tau, ncols=None):
    """Thin Q (M x ncols, default K) = Q I[:, :ncols]."""
    m = VR.shape[0]
    k = len(tau)
    ncols = k if ncols is None else ncols
    e = np.zeros((m, ncols), dtype=np.float64, order="F")
    e[np.arange(min(m, ncols)), np.arange(min(m, ncols))] = 1.0
    return apply_q(VR, tau, e)


def trsv_upper(R, B):
    """R^{-1} B for the upper triangle of the square R (back substitution)."""
    r = np.asfortranarray(R, dtype=np.float64)
    b = _fortran(B if B.ndim == 2 else B.reshape(-1, 1))
    n = r.shape[0]
    _load().oracle_trsv_upper(n, _p(r), max(1, n), b.shape[1], _p(b), max(1, n))
    return b


def lstsq(A, B):
    """Least-squares solution of A X = B for M >= N and full column rank:
    with A = QR, X = R^{-1} (Q^T B)[0:N] (the unique minimiser; Section 2.1's
    Q and R). Returns (X, Q^T B)."""
    M, N = A.shape
    VR, tau = geqr2(A)
    QtB = apply_qt(VR, tau, B)
    X = trsv_upper(np.asfortranarray(VR[:N, :N]), np.asfortranarray(QtB[:N]))
    return X, QtB


def larft(VR, tau, j0, k):
    """Compact-WY T (k x k, upper) of reflectors j0..j0+k-1."""
    v = np.asfortranarray(VR, dtype=np.float64)
    m = v.shape[0]
    t = np.zeros((k, k), dtype=np.float64, order="F")
    tt = np.ascontiguousarray(tau, dtype=np.float64)
    _load().oracle_larft(m, j0, k, _p(v), max(1, m), _p(tt), _p(t), max(1, k))
    return t


def gram_entry(A, i, j):
    a = np.asfortranarray(A, dtype=np.float64)
    return float(_load().oracle_gram_entry(a.shape[0], _p(a), max(1, a.shape[0]), i, j))


MLP_NPARAM = 8769


def mlp_forward(params, X):
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(X, dtype=np.float64)
    y = np.zeros(x.shape[0], dtype=np.float64)
    _load().oracle_mlp_forward(_p(p), _p(x), x.shape[0], _p(y))
    return y


def mlp_grad(params, X, y):
    """(loss, grad) of L = 1/(2n) sum (yhat - y)^2."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(X, dtype=np.float64)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(MLP_NPARAM, dtype=np.float64)
    loss = _load().oracle_mlp_grad(_p(p), _p(x), _p(yy), x.shape[0], _p(g))
    return float(loss), g


# ---------------------------------------------------------------------------
# Comparisons the method admits (R is unique only up to row signs).
# ---------------------------------------------------------------------------

def upper(VR):
    """The R factor (upper triangle / trapezoid) of a packed result."""
    m, n = VR.shape
    return np.triu(np.asarray(VR))[:min(m, n), :]


def sign_normalize(R):
    """D R with D = diag(sign(R_ii)), sign(0) = +1: rows flipped so that the
    diagonal is non-negative."""
    R = np.array(R, dtype=np.float64)
    k = min(R.shape)
    d = np.where(np.diag(R)[:k] < 0.0, -1.0, 1.0)
    R[:k, :] *= d[:, None]
    return R


def r_rel_diff(R_a, R_b):
    """||D_a R_a - D_b R_b||_F / ||R_b||_F."""
    a = sign_normalize(R_a)
    b = sign_normalize(R_b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def residual(A, Q, R):
    """||A - Q R||_F / ||A||_F."""
    na = np.linalg.norm(A)
    return float(np.linalg.norm(A - Q @ R) / (na if na > 0 else 1.0))


def orthogonality(Q):
    """||I - Q^T Q||_F."""
    k = Q.shape[1]
    return float(np.linalg.norm(np.eye(k) - Q.T @ Q))


def invariant_bound(M, N):
    """20 * K * eps with K = min(M, N)."""
    return 20.0 * min(M, N) * EPS
