"""Batched uneven-size tile QR: one persistent launch over the union of the
matrices' DAGs, captured in a hipGraph and replayed, against a loop of
per-matrix launches and against the CPU oracle.

Each tile task's arithmetic depends only on the tiles it reads, and the DAG
fixes the order in which a tile is updated, so replays of a launch give the
same bits whatever the schedule, and so does the per-matrix loop when it
runs the same register class. A batch runs every matrix in the class of its
largest tile order, whose panels use a narrower register micro-panel, so
across classes the results agree to rounding only; the oracle pins the
result itself."""
import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs
from helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


def _setup(shapes, seed, tilings):
    import torch
    import paper_1102_5328_amd as tq
    mats = inputs.batch_matrices(shapes, seed=seed)
    A0 = [to_dev(a) for a in mats]
    As = [to_dev(a) for a in mats]
    nbs = [t[0] for t in tilings]
    ibs = [t[1] for t in tilings]
    Ts = [torch.empty(max(1, tq.T_size(m, n, nb, ib)), dtype=torch.float64, device="cuda")
          for (m, n), nb, ib in zip(shapes, nbs, ibs)]
    return mats, A0, As, nbs, ibs, Ts


def _restore(As, A0):
    for a, a0 in zip(As, A0):
        a.copy_(a0)


def _tilings(shapes):
    import paper_1102_5328_amd as tq
    out = []
    for m, n in shapes:
        nb, ib, _ = tq.tune(m, n, len(shapes))
        out.append((nb, ib))
    return out


def _check_against_oracle(mats, As, idx):
    for b in idx:
        VR = to_host(As[b])
        VRo, _ = oracle.geqr2(mats[b])
        cond = np.linalg.cond(mats[b])
        r = oracle.r_rel_diff(oracle.upper(VR), oracle.upper(VRo))
        assert r <= 1e-10 * cond, (b, mats[b].shape, r)


def _rel(a, b):
    import torch
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def test_batched_small_mixed_tilings():
    """40 uneven matrices, three tile orders and several inner blocks in one
    launch: graph replays after eager work give the same bits, agree with
    the per-matrix loop to rounding, and every matrix matches the oracle."""
    import torch
    import paper_1102_5328_amd as tq
    shapes = inputs.batch_shapes(40, seed=3, m_lo=40, m_hi=400, n_lo=16)
    choices = [(64, 16), (64, 32), (96, 24), (96, 48), (128, 32), (128, 64), (128, 128), (64, 64)]
    tilings = [choices[b % len(choices)] for b in range(len(shapes))]
    mats, A0, As, nbs, ibs, Ts = _setup(shapes, 3, tilings)
    tq.factor_loop(As, nbs, ibs, Ts)
    tq.sync()
    loop = [a.clone() for a in As]
    first = None
    for rep in range(3):
        _restore(As, A0)
        torch.cuda.synchronize()
        tq.factor_batched(As, nbs, ibs, Ts)
        tq.sync()
        if first is None:
            first = [a.clone() for a in As]
        for b in range(len(As)):
            assert torch.equal(As[b], first[b]), (rep, b, shapes[b], tilings[b])
    for b in range(len(As)):
        assert _rel(As[b], loop[b]) < 1e-12, (b, shapes[b], tilings[b])
    _check_against_oracle(mats, As, range(len(As)))


def test_batched_same_class_matches_loop_bitwise():
    """All tile orders in one register class (NB <= 128, NB > 64): the batched
    launch and the per-matrix loop give the same bits."""
    import torch
    import paper_1102_5328_amd as tq
    shapes = inputs.batch_shapes(30, seed=4, m_lo=40, m_hi=500, n_lo=16)
    choices = [(96, 24), (128, 32), (128, 64), (96, 96), (128, 16)]
    tilings = [choices[b % len(choices)] for b in range(len(shapes))]
    mats, A0, As, nbs, ibs, Ts = _setup(shapes, 4, tilings)
    tq.factor_loop(As, nbs, ibs, Ts)
    tq.sync()
    loop = [a.clone() for a in As]
    _restore(As, A0)
    torch.cuda.synchronize()
    tq.factor_batched(As, nbs, ibs, Ts)
    tq.sync()
    for b in range(len(As)):
        assert torch.equal(As[b], loop[b]), (b, shapes[b], tilings[b])


def test_batched_config4_2000_matrices():
    """2000 matrices, M ~ U{64..1024}, N ~ U{32..M}, uniform[-1,1], seed 0,
    (NB, IB) per matrix from qr_tune with the batch count: two replays of the
    batched launch give the same bits and agree with the per-matrix loop to
    rounding (bit for bit when one register class covers every tile order);
    a sample of matrices against the oracle."""
    import torch
    import paper_1102_5328_amd as tq
    shapes = inputs.batch_shapes(2000, seed=0)
    tilings = _tilings(shapes)
    one_class = len({(nb > 64) for nb, _ in tilings}) == 1
    mats, A0, As, nbs, ibs, Ts = _setup(shapes, 0, tilings)
    tq.factor_loop(As, nbs, ibs, Ts)
    tq.sync()
    loop = [a.clone() for a in As]
    first = None
    for rep in range(2):
        _restore(As, A0)
        torch.cuda.synchronize()
        tq.factor_batched(As, nbs, ibs, Ts)
        tq.sync()
        if first is None:
            first = [a.clone() for a in As]
        bad = [b for b in range(len(As)) if not torch.equal(As[b], first[b])]
        assert not bad, (rep, bad[:10])
    if one_class:
        bad = [b for b in range(len(As)) if not torch.equal(As[b], loop[b])]
    else:
        bad = [b for b in range(len(As)) if _rel(As[b], loop[b]) >= 1e-12]
    assert not bad, (one_class, bad[:10])
    rng = np.random.default_rng(1)
    _check_against_oracle(mats, As, rng.choice(len(As), size=12, replace=False))


def test_batched_empty_and_degenerate():
    """An empty batch, empty matrices, and single rows/columns. Section 2.1's
    reflector of a zero-length tail is the identity (tau = 0), so a 1 x 1
    matrix and the row of a 1 x n matrix are left as they are."""
    import torch
    import paper_1102_5328_amd as tq
    tq.factor_batched([], [], [], [])
    shapes = [(0, 5), (5, 0), (1, 1), (70, 1), (1, 70)]
    As = []
    for m, n in shapes:
        t = tq.colmajor(m, n)
        t.fill_(0.5)
        As.append(t)
    Ts = [torch.empty(max(1, tq.T_size(m, n, 64, 16)), dtype=torch.float64, device="cuda")
          for m, n in shapes]
    tq.factor_batched(As, [64] * 5, [16] * 5, Ts)
    tq.sync()
    assert to_host(As[2])[0, 0] == 0.5
    # 70 x 1 with NB = 64: GEQRT on the first 64 rows, then TSQRT folds in
    # the last 6; R_00 is +-||a|| (the sign differs from one unblocked
    # reflector: R is unique up to row signs).
    assert abs(to_host(As[3])[0, 0]) == pytest.approx(0.5 * np.sqrt(70), rel=1e-14)
    np.testing.assert_array_equal(to_host(As[4])[0], 0.5)
