"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark. This module holds no QR arithmetic: it only draws random numbers,
so that the oracle and the HIP path can be fed the same bytes.

Matrices are FP64, column-major (numpy Fortran order, lda = M). A matrix is
drawn as ``rng.X(size=(N, M)).T`` so that the generator's stream fills
columns, i.e. the bytes in memory are the stream in order.
"""
import numpy as np


def uniform(M, N, seed=0, lo=-1.0, hi=1.0):
    """Entries iid uniform[lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(lo, hi, size=(N, M)).T)


def normal(M, N, seed=0):
    """Entries iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal(size=(N, M)).T)


def ill_conditioned(N, seed=0, log10_cond=12.0):
    """A = U diag(logspace(0, -log10_cond, N)) V^T, with U and V the Q factors
    of two N(0,1) matrices drawn in that order from one generator. The
    library QR here is only a generator of random orthogonal matrices."""
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal(size=(N, N)).T
    G2 = rng.standard_normal(size=(N, N)).T
    U, _ = np.linalg.qr(G1)
    V, _ = np.linalg.qr(G2)
    s = np.logspace(0.0, -log10_cond, N)
    return np.asfortranarray((U * s[None, :]) @ V.T)


def batch_shapes(count=2000, seed=0, m_lo=64, m_hi=1024, n_lo=32):
    """Uneven batch: M_b ~ U{m_lo..m_hi}, N_b ~ U{n_lo..M_b}."""
    rng = np.random.default_rng(seed)
    Ms = rng.integers(m_lo, m_hi + 1, size=count)
    Ns = np.array([rng.integers(n_lo, m + 1) for m in Ms])
    return [(int(m), int(n)) for m, n in zip(Ms, Ns)]


def batch_matrices(shapes, seed=0):
    """Entries iid uniform[-1, 1] for each (M, N) of `shapes`, one stream."""
    rng = np.random.default_rng(seed + 1)
    return [np.asfortranarray(rng.uniform(-1.0, 1.0, size=(n, m)).T) for m, n in shapes]


def log_uniform_shapes(count, seed, lo=256, hi=32768):
    """(M, N) with M and N independently log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    lm = rng.uniform(np.log(lo), np.log(hi), size=count)
    ln = rng.uniform(np.log(lo), np.log(hi), size=count)
    return [(int(round(np.exp(a))), int(round(np.exp(b)))) for a, b in zip(lm, ln)]


def torch_normal(M, N, seed=0, device="cuda"):
    """N(0,1) matrix generated directly on the device (large benchmark
    inputs), column-major: returned as the transpose view of an N x M
    contiguous tensor, i.e. a column-major M x N matrix with lda = M."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.randn((N, M), dtype=torch.float64, device=device, generator=g)
    return t.t()


def torch_uniform(M, N, seed=0, device="cuda", lo=-1.0, hi=1.0):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.rand((N, M), dtype=torch.float64, device=device, generator=g)
    t.mul_(hi - lo).add_(lo)
    return t.t()
