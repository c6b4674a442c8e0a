"""Host checks of the test helpers that set tolerances (CPU only)."""
import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs
from helpers import cond_estimate


@pytest.mark.parametrize("M,N", [(300, 300), (500, 120), (120, 400)])
def test_cond_estimate_matches_svd(M, N):
    A = inputs.normal(M, N, seed=4)
    VR, _ = oracle.geqr2(A)
    R = oracle.upper(VR)
    est = cond_estimate(R, iters=60)
    if M >= N:
        exact = np.linalg.cond(A)
    else:  # wide: the tolerance uses sigma_max(A) / sigma_min(R[:, :K])
        s = np.linalg.svd(A, compute_uv=False)
        exact = s[0] / np.linalg.svd(R[:, :M], compute_uv=False)[-1]
    assert est == pytest.approx(exact, rel=0.05)


def test_cond_estimate_ill_conditioned():
    A = inputs.ill_conditioned(200, seed=0, log10_cond=8.0)
    VR, _ = oracle.geqr2(A)
    est = cond_estimate(oracle.upper(VR), iters=80)
    assert 0.5e8 <= est <= 2e8
