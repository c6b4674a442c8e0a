"""qr_factor_noalloc (the allocation-free variant of qr_factor) against
qr_factor through the C ABI: on the same input both give bit-identical A
(R and the reflectors) and T, since every tile sees the same sequence of
kernel operations whatever the ticket order. Two calls in a row, the second
on a smaller matrix (the static scratch keeps the first call's contents).
The size limit is checked on the host before any device call (see
test_library_host.py)."""
import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs
from paper_1102_5328_amd._lib import TileQRError

pytestmark = pytest.mark.gpu


def _pair(M, N, nb, ib, seed):
    import torch
    import paper_1102_5328_amd as tq
    A = inputs.uniform(M, N, seed=seed)
    outs = []
    for noalloc in (False, True):
        dA = tq.colmajor(M, N)
        dA.copy_(torch.from_numpy(A))
        T = torch.full((max(1, tq.T_size(M, N, nb, ib)),), float("nan"), dtype=torch.float64,
                       device="cuda")
        if noalloc:
            tq.factor_noalloc(dA, nb, ib, T)
        else:
            tq.factor(dA, nb, ib, T)
        tq.sync()
        outs.append((dA.cpu().numpy(), T.cpu().numpy()))
    return A, outs


@pytest.mark.parametrize("calls", [[(700, 520, 128, 32, 1), (300, 200, 64, 16, 2)]])
def test_noalloc_matches_qr_factor(calls):
    for M, N, nb, ib, seed in calls:
        A, ((Ar, Tr), (An, Tn)) = _pair(M, N, nb, ib, seed)
        print("M=%d N=%d nb=%d ib=%d" % (M, N, nb, ib), flush=True)
        assert np.array_equal(Ar, An)
        K = min(M, N)
        # T: compare where qr_factor wrote it (the rest of the buffer is unused)
        wr = ~np.isnan(Tr)
        assert np.array_equal(np.isnan(Tn), ~wr)
        assert np.array_equal(Tr[wr], Tn[wr])
        # and the result is a QR factorization of A (oracle R)
        VRo, _ = oracle.geqr2(A)
        r_rel = oracle.r_rel_diff(oracle.upper(An)[:K], oracle.upper(VRo)[:K])
        assert r_rel <= 1e-10 * np.linalg.cond(A)
