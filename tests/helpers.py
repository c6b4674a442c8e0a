"""Shared helpers of the GPU tests: moving column-major matrices between
numpy and the device, and the checks the method admits (R up to row signs,
Q^T A upper triangular, orthogonality of Q)."""
import numpy as np

import oracle


def to_dev(A, extra_ld=0):
    """Column-major device copy of a numpy matrix (lda = M + extra_ld)."""
    import torch
    M, N = A.shape
    buf = torch.empty((max(N, 1), M + extra_ld), dtype=torch.float64, device="cuda")
    t = buf.t()[:M]
    t.copy_(torch.from_numpy(np.asfortranarray(A)))
    return t


def to_host(t):
    return np.asfortranarray(t.detach().cpu().numpy())


def factor_gpu(A, nb, ib, extra_ld=0, units=None, p=None):
    """Factor a numpy matrix on the GPU, on a grid sized for `units` compute
    units (None: all of them); p: row domains of qr_factor_ca (None:
    qr_factor). Returns (VR host, T device, A dev)."""
    import paper_1102_5328_amd as tq
    import torch
    dA = to_dev(A, extra_ld)
    with grid_units(units):
        if p is None:
            _, T, _, _ = tq.factor(dA, nb, ib)
        else:
            _, T = tq.factor_ca(dA, nb, ib, p)
        tq.sync()
    torch.cuda.synchronize()
    return to_host(dA), T, dA


def apply_qt_gpu(dA, T, nb, ib, B, p=None):
    import paper_1102_5328_amd as tq
    dB = to_dev(B)
    if p is None:
        tq.apply_Qt(dA, T, nb, ib, dB)
    else:
        tq.apply_Qt_ca(dA, T, nb, ib, p, dB)
    tq.sync()
    return to_host(dB)


def check_factorization(A, nb, ib, extra_ld=0, cond=None, full_orth=True, units=None, p=None):
    """Factor A on the GPU (grid sized for `units` compute units, None: all;
    p row domains, None: the flat qr_factor) and check it against the oracle
    and the invariants. Returns a dict of the measured quantities."""
    M, N = A.shape
    K = min(M, N)
    VR, T, dA = factor_gpu(A, nb, ib, extra_ld, units, p)
    VRo, tauo = oracle.geqr2(A)
    R_g, R_o = oracle.upper(VR), oracle.upper(VRo)
    out = {}
    out["r_rel"] = oracle.r_rel_diff(R_g, R_o)
    if cond is None:
        cond = np.linalg.cond(A) if K > 0 else 1.0
    out["r_bound"] = 1e-10 * cond
    bound = oracle.invariant_bound(M, N)
    nA = np.linalg.norm(A)
    # ||A - QR|| / ||A|| = ||Q^T A - [R; 0]|| / ||A|| for orthogonal Q.
    E = apply_qt_gpu(dA, T, nb, ib, A, p)
    E[:K] -= R_g
    out["residual"] = np.linalg.norm(E) / nA if nA > 0 else 0.0
    if full_orth:
        Qt = apply_qt_gpu(dA, T, nb, ib, np.eye(M), p)
        out["orth"] = np.linalg.norm(np.eye(M) - Qt @ Qt.T)
    out["bound"] = bound
    return out


class grid_units:
    """Context manager: size the persistent grid for `cus` compute units
    (None: the device's count, i.e. the full grid; 0: the decision table's
    choice for the shape), restoring "no setting" on exit, so a test's grid
    never depends on what ran before it."""

    def __init__(self, cus):
        self.cus = cus

    def __enter__(self):
        import paper_1102_5328_amd as tq
        import torch
        cus = self.cus
        if cus is None:
            cus = torch.cuda.get_device_properties(0).multi_processor_count
        tq.set_compute_units(cus)
        return cus

    def __exit__(self, *exc):
        import paper_1102_5328_amd as tq
        tq.set_compute_units(0)
        return False


def cond_estimate(R, iters=30, seed=0):
    """2-norm condition number of an upper-triangular (or trapezoidal) R by
    power iteration on R^T R for sigma_max and inverse iteration (two
    triangular solves per step) for sigma_min; R has the singular values of
    A. Used only to set the 1e-10 * cond(A) tolerance at sizes where a full
    SVD is too slow."""
    import scipy.linalg as sl
    K = min(R.shape)
    Rk = np.ascontiguousarray(R[:K, :K]) if R.shape[1] >= K else R
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(Rk.shape[1])
    smax = 0.0
    for _ in range(iters):
        y = Rk.T @ (Rk @ x)
        smax = np.sqrt(np.linalg.norm(y) / np.linalg.norm(x))
        x = y / np.linalg.norm(y)
    if R.shape[1] > K:  # wide: sigma_max over all columns, sigma_min of the square part
        x = rng.standard_normal(R.shape[1])
        for _ in range(iters):
            y = R.T @ (R @ x)
            smax = max(smax, np.sqrt(np.linalg.norm(y) / np.linalg.norm(x)))
            x = y / np.linalg.norm(y)
    x = rng.standard_normal(K)
    smin_inv = 0.0
    for _ in range(iters):
        z = sl.solve_triangular(Rk, x, lower=False)
        y = sl.solve_triangular(Rk, z, lower=False, trans="T")
        smin_inv = np.sqrt(np.linalg.norm(y) / np.linalg.norm(x))
        x = y / np.linalg.norm(y)
    return float(smax * smin_inv)
