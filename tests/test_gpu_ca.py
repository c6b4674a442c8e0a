"""GPU parity of the communication-avoiding tile QR (qr_factor_ca /
qr_apply_Qt_ca: the tile rows in p domains, each reduced by its own
GEQRT + TSQRT chain, the domains' R factors merged pairwise over a binary
tree; Section 7) against the CPU oracle on the same seeded inputs. R is
unique up to row signs for a full-rank matrix whatever the reduction order,
so the oracle's Householder QR is the reference:
  * R after row-sign normalisation within 1e-10 * cond(A);
  * ||Q^T A - [R; 0]|| / ||A|| and ||I - Q^T Q|| within 20 K eps (Q^T from
    qr_apply_Qt_ca applied to A and to the identity).
Covers one and several tile rows per domain, a ragged last domain (its head
tile shorter than NB, merged as a trapezoid), every row-wave class (NB <=
128, 256, 512), inner blocks that do not divide NB or are wider than a
register panel, wide matrices (M < N), and p = 1 giving qr_factor's results
bit for bit."""
import numpy as np
import pytest

from paper_1102_5328_amd import inputs
from helpers import check_factorization, grid_units, to_dev, to_host

pytestmark = pytest.mark.gpu


def _assert_ok(r):
    assert r["r_rel"] <= r["r_bound"], r
    assert r["residual"] <= r["bound"], r
    if "orth" in r:
        assert r["orth"] <= r["bound"], r


@pytest.mark.parametrize("M,N,nb,ib,p", [
    (1000, 200, 64, 16, 2),     # 16 tile rows in two domains of 8
    (1000, 200, 64, 16, 5),     # domains of 4, a ragged last one
    (1000, 200, 64, 16, 16),    # one tile row per domain: the tree alone
    (1000, 200, 64, 16, 100),   # p > MT is taken as MT
    (700, 150, 128, 32, 3),     # ragged last tile row as a domain of its own
    (450, 130, 64, 12, 3),      # IB does not divide NB
    (900, 300, 96, 48, 4),      # NB = 96
    (600, 600, 64, 16, 4),      # square: the tree on every panel
    (300, 700, 64, 32, 3),      # wide: M < N
    (1300, 256, 256, 32, 3),    # two row waves per column group
    (1100, 300, 512, 64, 2),    # four row waves
    (700, 200, 128, 128, 3),    # IB = NB wider than the register panel
])
def test_ca_factor_matches_oracle(M, N, nb, ib, p):
    A = inputs.uniform(M, N, seed=M * 7 + N + p)
    r = check_factorization(A, nb, ib, p=p)
    print((M, N, nb, ib, p), r)
    _assert_ok(r)


@pytest.mark.parametrize("units", [None, 8])
def test_ca_on_full_and_small_grid(units):
    """The same factorization on the full grid and on a grid of 8 compute
    units (16 workgroups taking the tickets of a 64-domain tree)."""
    A = inputs.normal(4096, 128, seed=11)
    r = check_factorization(A, 64, 16, units=units, p=64, full_orth=False)
    print(units, r)
    _assert_ok(r)


def test_ca_p1_is_the_flat_factorization():
    """p = 1 runs the flat tree's DAG: A and T bit-identical to qr_factor."""
    import paper_1102_5328_amd as tq
    import torch
    A = inputs.normal(700, 300, seed=5)
    n = tq.T_size(700, 300, 64, 16)
    assert n == tq.T_size(700, 300, 64, 16, 1)
    # zero-filled: the T slots of tiles above the diagonal are never written
    T1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    T2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    with grid_units(None):
        d1 = to_dev(A)
        tq.factor(d1, 64, 16, T1)
        d2 = to_dev(A)
        tq.factor_ca(d2, 64, 16, 1, T2)
        tq.sync()
    torch.cuda.synchronize()
    assert np.array_equal(to_host(d1), to_host(d2))
    assert torch.equal(T1, T2)


def test_ca_replays_are_identical():
    """Two runs of a tree factorization give the same bits (the reduction
    order is fixed by the tree, not by the schedule)."""
    import paper_1102_5328_amd as tq
    import torch
    A = inputs.normal(2000, 256, seed=9)
    outs = []
    with grid_units(None):
        for _ in range(2):
            d = to_dev(A)
            T = torch.zeros(tq.T_size(2000, 256, 64, 16, 8), dtype=torch.float64, device="cuda")
            tq.factor_ca(d, 64, 16, 8, T)
            tq.sync()
            outs.append((to_host(d), T.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
