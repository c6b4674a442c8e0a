"""Tile QR at full size, in the launch configuration the benchmark times
(the tiling qr_tune gives once the shipped decision table is loaded), on
properties that hold at any size and that the oracle can check entry by
entry:
  * column norms: ||R[:, j]|| = ||A[:, j]|| (Q is orthogonal);
  * sampled Gram entries: (R^T R)_ij = (A^T A)_ij, the right side computed
    by the oracle from the two columns;
  * residual on sampled columns, ||Q^T a_j - r_j|| / ||a_j||, through
    qr_apply_Qt;
  * a randomized orthogonality sketch: for Gaussian X (M x 8), Y = Q^T X,
    ||X^T X - Y^T Y||_F / ||X||_F^2 (E||E g||^2 = ||E||_F^2).
Tolerances are the invariants' 20 * K * eps (Frobenius), with K = min(M, N).
"""
import os

import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1102_5328_amd", "tuning", "decision_table.txt")


def _tiling(M, N):
    import paper_1102_5328_amd as tq
    if os.path.exists(TABLE):
        tq.tune_load(TABLE)
    nb, ib, _ = tq.tune(M, N, 1)
    return nb, ib


def _properties(A0, nb, ib, nsample=16, seed=0):
    import torch
    import paper_1102_5328_amd as tq
    M, N = A0.shape
    K = min(M, N)
    bound = oracle.invariant_bound(M, N)
    A = tq.colmajor(M, N)
    A.copy_(A0)
    _, T, _, _ = tq.factor(A, nb, ib)
    tq.sync()
    R = torch.triu(A[:K])
    # Column norms (all columns, on the device).
    na = torch.linalg.vector_norm(A0, dim=0)
    nr = torch.linalg.vector_norm(R, dim=0)
    colerr = float(torch.max(torch.abs(nr - na) / na))
    assert colerr <= bound, ("column norms", colerr, bound)
    rng = np.random.default_rng(seed)
    cols = np.sort(rng.choice(N, size=min(nsample, N), replace=False))
    # Gram entries against the oracle.
    for _ in range(nsample):
        i, j = sorted(rng.integers(0, N, size=2).tolist())
        k = min(i, j, K - 1) + 1
        rtr = float(torch.dot(R[:k, i], R[:k, j]))
        two = torch.stack([A0[:, i], A0[:, j]], dim=1).cpu().numpy()
        ata = oracle.gram_entry(np.asfortranarray(two), 0, 1)
        scale = float(na[i] * na[j])
        assert abs(rtr - ata) <= bound * scale, ("gram", i, j, rtr, ata)
    # Residual on sampled columns.
    B = tq.colmajor(M, len(cols))
    B.copy_(A0[:, torch.as_tensor(cols, device="cuda")])
    tq.apply_Qt(A, T, nb, ib, B)
    tq.sync()
    Rc = R[:, torch.as_tensor(cols, device="cuda")]
    E = B.clone()
    E[:K] -= Rc
    res = float(torch.linalg.norm(E) / torch.linalg.norm(A0[:, torch.as_tensor(cols, device="cuda")]))
    assert res <= bound, ("residual", res, bound)
    # Orthogonality sketch.
    g = torch.Generator(device="cuda")
    g.manual_seed(seed + 7)
    X = torch.randn((8, M), dtype=torch.float64, device="cuda", generator=g).t()
    Y = tq.colmajor(M, 8)
    Y.copy_(X)
    tq.apply_Qt(A, T, nb, ib, Y)
    tq.sync()
    orth = float(torch.linalg.norm(X.t() @ X - Y.t() @ Y) / torch.linalg.norm(X) ** 2)
    assert orth <= bound, ("orthogonality sketch", orth, bound)
    return {"colerr": colerr, "residual": res, "orth": orth, "bound": bound}


def test_square_16384_benchmark_configuration():
    M = N = 16384
    nb, ib = _tiling(M, N)
    A0 = inputs.torch_normal(M, N, seed=0)
    r = _properties(A0, nb, ib)
    print("16384", nb, ib, r)


@pytest.mark.parametrize("M,N", [(65536, 256), (65536, 1024), (16384, 4096)])
def test_tall_configurations(M, N):
    nb, ib = _tiling(M, N)
    A0 = inputs.torch_normal(M, N, seed=0)
    r = _properties(A0, nb, ib)
    print((M, N), nb, ib, r)


def test_wide_8192x2048_transposed():
    """Wide shape (M < N): K = M reflectors, R is an M x N trapezoid."""
    M, N = 2048, 8192
    nb, ib = _tiling(M, N)
    A0 = inputs.torch_normal(M, N, seed=1)
    r = _properties(A0, nb, ib)
    print((M, N), nb, ib, r)


def test_ill_conditioned_4096():
    """A = U diag(logspace(0, -12, N)) V^T: the R comparison bound
    1e-10 * cond is vacuous here, the invariants carry the case."""
    import torch
    N = 4096
    nb, ib = _tiling(N, N)
    A = inputs.ill_conditioned(N, seed=0)
    A0 = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    r = _properties(A0, nb, ib)
    print("illcond", nb, ib, r)
