"""GPU parity of what is built on the stored reflectors (V, T): B <- Q B
(qr_apply_Q_ca), the explicit Q (qr_form_Q_ca) and least squares
(qr_solve_ls_ca), for the flat tree and the communication-avoiding tree,
against the CPU oracle on the same seeded inputs:
  * Q Q^T B = B (the Q application is the exact inverse of the Q^T one);
  * the first N columns of Q equal the oracle's after the column signs of
    R's diagonal are normalised (they are unique up to those signs), and
    Q[:, :N] R = A;
  * the full Q (k = M) is orthogonal;
  * the least-squares X equals the oracle's (unique for a full-rank A), and
    the norm of rows N.. of the returned Q^T B is the residual norm.
Tolerances: 20 K eps relative for invariants, 1e-10 cond(A) for X and Q."""
import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs
from helpers import grid_units, to_dev, to_host

pytestmark = pytest.mark.gpu


def _factor(A, nb, ib, p):
    import paper_1102_5328_amd as tq
    dA = to_dev(A)
    with grid_units(None):
        _, T = tq.factor_ca(dA, nb, ib, p)
        tq.sync()
    return dA, T


@pytest.mark.parametrize("M,N,nb,ib,p", [
    (300, 200, 64, 16, 1),
    (700, 150, 128, 32, 3),
    (450, 430, 64, 12, 1),
    (520, 200, 256, 32, 1),
    (1000, 120, 64, 16, 16),
])
def test_apply_Q_inverts_apply_Qt(M, N, nb, ib, p):
    import paper_1102_5328_amd as tq
    A = inputs.uniform(M, N, seed=M + N)
    B = inputs.normal(M, 7, seed=3)
    dA, T = _factor(A, nb, ib, p)
    dB = to_dev(B)
    tq.apply_Qt_ca(dA, T, nb, ib, p, dB)
    tq.apply_Q(dA, T, nb, ib, dB, p=p)
    tq.sync()
    err = np.linalg.norm(to_host(dB) - B) / np.linalg.norm(B)
    assert err <= oracle.invariant_bound(M, N), err


@pytest.mark.parametrize("M,N,nb,ib,p", [
    (300, 200, 64, 16, 1),
    (700, 150, 128, 32, 3),
    (257, 257, 128, 48, 1),
    (600, 100, 512, 64, 1),
])
def test_form_Q_matches_oracle(M, N, nb, ib, p):
    import paper_1102_5328_amd as tq
    A = inputs.uniform(M, N, seed=2 * M + N)
    K = min(M, N)
    dA, T = _factor(A, nb, ib, p)
    Q = to_host(tq.form_Q(dA, T, nb, ib, k=K, p=p))
    tq.sync()
    VR = to_host(dA)
    R = oracle.upper(VR)[:K]
    VRo, tauo = oracle.geqr2(A)
    Qo = oracle.form_q(VRo, tauo, K)
    Ro = oracle.upper(VRo)[:K]
    d, do = np.sign(np.diag(R)), np.sign(np.diag(Ro))
    cond = np.linalg.cond(A)
    assert np.linalg.norm(Q * d - Qo * do) / np.sqrt(K) <= 1e-10 * cond
    bound = oracle.invariant_bound(M, N)
    assert np.linalg.norm(Q @ R - A) / np.linalg.norm(A) <= bound


@pytest.mark.parametrize("M,N,nb,ib,p", [(300, 200, 64, 16, 1), (700, 150, 128, 32, 3)])
def test_full_Q_is_orthogonal(M, N, nb, ib, p):
    import paper_1102_5328_amd as tq
    A = inputs.normal(M, N, seed=7)
    dA, T = _factor(A, nb, ib, p)
    Q = to_host(tq.form_Q(dA, T, nb, ib, k=M, p=p))
    tq.sync()
    assert np.linalg.norm(Q.T @ Q - np.eye(M)) <= oracle.invariant_bound(M, N)


@pytest.mark.parametrize("M,N,nb,ib,p,nrhs", [
    (300, 200, 64, 16, 1, 3),
    (1000, 120, 64, 16, 16, 1),
    (700, 150, 128, 32, 3, 5),
    (256, 256, 128, 16, 1, 2),   # square: the solve of A X = B
])
def test_least_squares_matches_oracle(M, N, nb, ib, p, nrhs):
    import paper_1102_5328_amd as tq
    A = inputs.normal(M, N, seed=M * 3 + N)
    B = inputs.normal(M, nrhs, seed=11)
    dA, T = _factor(A, nb, ib, p)
    dB = to_dev(B)
    tq.solve_ls(dA, T, nb, ib, dB, p=p)
    tq.sync()
    out = to_host(dB)
    X = out[:N]
    Xo, _ = oracle.lstsq(A, B)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-10 * cond
    res = np.linalg.norm(A @ X - B, axis=0)
    if M > N:
        np.testing.assert_allclose(np.linalg.norm(out[N:], axis=0), res, rtol=1e-8)
