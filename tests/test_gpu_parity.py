"""GPU parity of the tile QR (HIP path through the C ABI) against the CPU
oracle on the same seeded inputs: R after row-sign normalisation within
1e-10 * cond(A), ||A - QR||/||A|| and ||I - Q^T Q|| within 20 * K * eps, and
the single-tile special case where the reflectors themselves must match."""
import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs
from helpers import check_factorization, factor_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

# Tile orders above 128 run the same kernels with two or four row waves per
# column group (128-row slabs per wave).


def _assert_ok(r):
    assert r["r_rel"] <= r["r_bound"], r
    assert r["residual"] <= r["bound"], r
    if "orth" in r:
        assert r["orth"] <= r["bound"], r


@pytest.mark.parametrize("units", [None, 16, 1])
def test_config1_512_nb128_ib32(units):
    """Configuration 1: M = N = 512, NB = 128, IB = 32, uniform[-1,1], seed 0,
    on the full grid, on 16 compute units, and on a single one (two
    workgroups take every task in ticket order)."""
    A = inputs.uniform(512, 512, seed=0)
    r = check_factorization(A, 128, 32, units=units)
    print("config1", units, r)
    _assert_ok(r)


@pytest.mark.parametrize("M,N,nb,ib", [
    (200, 200, 64, 16),     # ragged last tile, 4x4 tiles
    (300, 170, 64, 32),     # tall, ragged both ways
    (170, 300, 64, 32),     # wide (M < N)
    (257, 257, 128, 48),    # IB > 16: micro-panels + T assembly; IB does not divide NB
    (130, 97, 96, 24),      # NB = 96, IB = 24
    (384, 384, 128, 128),   # IB = NB
    (100, 100, 64, 5),      # odd IB
    (64, 512, 64, 16),      # one tile row
    (700, 64, 64, 64),      # one tile column (the TSQRT chain only)
    (33, 33, 16, 1),        # IB = 1
    (520, 520, 256, 32),    # two row waves per column group
    (600, 600, 512, 64),    # four row waves
    (450, 430, 192, 96),    # IB wider than the 32-column register panel
    (530, 300, 384, 384),   # IB = NB = 384, T assembled over 16-column panels
])
def test_factor_shapes(M, N, nb, ib):
    A = inputs.uniform(M, N, seed=M * 7 + N)
    r = check_factorization(A, nb, ib)
    print((M, N, nb, ib), r)
    _assert_ok(r)


def test_leading_dimension_padding():
    A = inputs.normal(150, 120, seed=3)
    r = check_factorization(A, 64, 16, extra_ld=13)
    _assert_ok(r)


@pytest.mark.parametrize("M,N,nb,ib", [(128, 16, 128, 16), (128, 8, 128, 8), (100, 16, 128, 16),
                                       (64, 16, 64, 16), (70, 12, 128, 12),
                                       (64, 64, 64, 16), (100, 60, 128, 32), (50, 90, 64, 24),
                                       (128, 128, 128, 128),
                                       (256, 200, 256, 48), (512, 100, 512, 128)])
def test_single_tile_reflectors_match_oracle(M, N, nb, ib):
    """M, N <= NB: qr_factor is one DGEQRT, so V and tau = diag(T_s) equal the
    unblocked oracle's reflectors up to rounding, for any IB."""
    A = inputs.normal(M, N, seed=21)
    VR, T, _ = factor_gpu(A, nb, ib)
    VRo, tauo = oracle.geqr2(A)
    K = min(M, N)
    np.testing.assert_allclose(VR, VRo, rtol=0, atol=1e-12 * np.abs(VRo).max())
    Th = T.cpu().numpy()
    tau = []
    for s in range(0, K, ib):
        blk = Th[s * ib:(s + min(ib, K - s)) * ib].reshape(-1, ib)  # columns of ld ib
        for c in range(min(ib, K - s)):
            tau.append(blk[c, c])
    np.testing.assert_allclose(tau, tauo, rtol=1e-12, atol=1e-14)


def test_ill_conditioned_invariants():
    """cond = 1e12: the R bound is vacuous, the invariants carry the check."""
    A = inputs.ill_conditioned(256, seed=0)
    r = check_factorization(A, 64, 16, cond=1e12)
    _assert_ok(r)


@pytest.mark.parametrize("M,N,nb,ib", [(300, 200, 64, 16), (384, 320, 128, 16)])
def test_power_of_two_scaling_is_exact(M, N, nb, ib):
    """The kernels form each reflector from the unscaled norm of its column
    (the range stated in tileqr.h). For s = 2^(+-400), about 1e(+-120), every
    operation scales exactly, so R(sA) = s R(A) and the reflectors are
    unchanged, bit for bit."""
    A = inputs.normal(M, N, seed=23)
    VR, _, _ = factor_gpu(A, nb, ib, units=16)
    for e in (400, -400):
        s = 2.0 ** e
        VRs, _, _ = factor_gpu(A * s, nb, ib, units=16)
        np.testing.assert_array_equal(oracle.upper(VRs), oracle.upper(VR) * s)
        np.testing.assert_array_equal(np.tril(VRs, -1), np.tril(VR, -1))
