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


def factor_gpu(A, nb, ib, extra_ld=0):
    """Factor a numpy matrix on the GPU. Returns (VR host, T device, A dev)."""
    import paper_1102_5328_amd as tq
    import torch
    dA = to_dev(A, extra_ld)
    _, T, _, _ = tq.factor(dA, nb, ib)
    tq.sync()
    torch.cuda.synchronize()
    return to_host(dA), T, dA


def apply_qt_gpu(dA, T, nb, ib, B):
    import paper_1102_5328_amd as tq
    dB = to_dev(B)
    tq.apply_Qt(dA, T, nb, ib, dB)
    tq.sync()
    return to_host(dB)


def check_factorization(A, nb, ib, extra_ld=0, cond=None, full_orth=True):
    """Factor A on the GPU and check it against the oracle and the invariants.
    Returns a dict of the measured quantities."""
    M, N = A.shape
    K = min(M, N)
    VR, T, dA = factor_gpu(A, nb, ib, extra_ld)
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
    E = apply_qt_gpu(dA, T, nb, ib, A)
    E[:K] -= R_g
    out["residual"] = np.linalg.norm(E) / nA if nA > 0 else 0.0
    if full_orth:
        Qt = apply_qt_gpu(dA, T, nb, ib, np.eye(M))
        out["orth"] = np.linalg.norm(np.eye(M) - Qt @ Qt.T)
    out["bound"] = bound
    return out
