"""The four tile kernels one at a time through qr_tile_task (Section 2.1),
against the oracle on the same seeded inputs:
  DGEQRT(k)      tile (k,k): R, the unit-lower V and tau = diag(T_s) equal
                 unblocked Householder QR of the tile;
  DLARFB(k,j)    A_kj <- Q_kk^T A_kj equals the oracle applying the tile's
                 reflectors one at a time;
  DTSQRT(i,k)    [R_kk; A_ik] -> R_kk, V_ik equals unblocked QR of the
                 stacked (NB + mb) x NB matrix, whose reflectors are
                 [e_j; 0; u_j] (the zeros of the triangle are preserved);
  DSSRFB(i,j,k)  [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij] equals the oracle
                 applying the stacked reflectors.
Every expected value comes from the oracle alone (the tile's QR, then the
stacked QR of the oracle's R); the GPU runs the same chain of tasks."""
import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs
from helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _tau_from_T(T, nb, ib, ncols, tile_off):
    """diag of the T_s blocks of one tile: column c of the tile's T block
    holds T_s's column c - s with its diagonal at row c - s."""
    t = T[tile_off:tile_off + ib * nb].reshape(nb, ib).T  # [row][col], ld = ib
    return np.array([t[c % ib, c] for c in range(ncols)])


@pytest.mark.parametrize("nb,ib,mlast", [(64, 16, 64), (128, 32, 128), (64, 12, 37), (128, 48, 90)])
def test_tile_kernels_against_oracle(nb, ib, mlast):
    import torch
    import paper_1102_5328_amd as tq
    # Three tile rows (the last one mlast rows), two tile columns.
    M, N = 2 * nb + mlast, 2 * nb
    A = inputs.uniform(M, N, seed=nb + ib + mlast)
    dA = to_dev(A)
    T = torch.zeros(tq.T_size(M, N, nb, ib), dtype=torch.float64, device="cuda")
    MT = 3
    k, j = 0, 1
    # --- oracle chain ----------------------------------------------------
    Akk = A[:nb, :nb]
    VRk, tauk = oracle.geqr2(Akk)
    Rk = np.triu(VRk)
    C_top = oracle.apply_qt(VRk, tauk, A[:nb, nb:2 * nb])          # LARFB(0,1)
    exp = {}
    Rcur, Ccur = Rk.copy(), C_top.copy()
    for i in (1, 2):
        rows = slice(i * nb, min((i + 1) * nb, M))
        S = np.vstack([Rcur, A[rows, :nb]])
        VRs, taus = oracle.geqr2(S)                                   # TSQRT(i,0)
        B = np.vstack([Ccur, A[rows, nb:2 * nb]])
        Bq = oracle.apply_qt(VRs, taus, B)                            # SSRFB(i,1,0)
        exp[i] = (VRs, taus, Bq)
        Rcur = np.triu(VRs[:nb])
        Ccur = Bq[:nb]
    # --- GPU chain: GEQRT(0), LARFB(0,1), TSQRT(1,0), SSRFB(1,1,0), TSQRT(2,0), SSRFB(2,1,0)
    tq.tile_task(0, dA, nb, ib, T, 0, 0, k)
    tq.sync()
    g = to_host(dA)
    assert _rel(np.triu(g[:nb, :nb]), Rk) < TOL
    assert _rel(np.tril(g[:nb, :nb], -1), np.tril(VRk, -1)) < TOL
    Th = T.cpu().numpy()
    assert _rel(_tau_from_T(Th, nb, ib, nb, 0), tauk) < TOL
    tq.tile_task(2, dA, nb, ib, T, 0, j, k)
    tq.sync()
    g = to_host(dA)
    assert _rel(g[:nb, nb:2 * nb], C_top) < TOL
    for i in (1, 2):
        rows = slice(i * nb, min((i + 1) * nb, M))
        mb = rows.stop - rows.start
        VRs, taus, Bq = exp[i]
        tq.tile_task(1, dA, nb, ib, T, i, 0, k)
        tq.sync()
        g = to_host(dA)
        assert _rel(np.triu(g[:nb, :nb]), np.triu(VRs[:nb])) < TOL, ("TSQRT R", i)
        # Reflectors: [e_j; 0; u_j]; the oracle's u_j are rows nb.. of its V.
        assert _rel(g[rows, :nb], VRs[nb:nb + mb]) < TOL, ("TSQRT V", i)
        # The oracle's reflectors keep the zeros of the triangle.
        assert np.all(np.tril(VRs[:nb], -1) == 0.0)
        Th = T.cpu().numpy()
        assert _rel(_tau_from_T(Th, nb, ib, nb, (k * MT + i) * ib * nb), taus) < TOL, ("tau", i)
        tq.tile_task(3, dA, nb, ib, T, i, j, k)
        tq.sync()
        g = to_host(dA)
        assert _rel(g[:nb, nb:2 * nb], Bq[:nb]) < TOL, ("SSRFB top", i)
        assert _rel(g[rows, nb:2 * nb], Bq[nb:nb + mb]) < TOL, ("SSRFB bottom", i)


def test_tile_task_argument_errors():
    import torch
    import paper_1102_5328_amd as tq
    from paper_1102_5328_amd import _lib
    dA = to_dev(np.ones((200, 130)))
    T = torch.zeros(tq.T_size(200, 130, 64, 16), dtype=torch.float64, device="cuda")
    f = _lib.lib().qr_tile_task
    import ctypes
    a, t = ctypes.c_void_p(dA.data_ptr()), ctypes.c_void_p(T.data_ptr())
    assert f(4, a, 200, 130, 200, 64, 16, t, 0, 0, 0, None) == -1
    assert f(1, a, 200, 130, 200, 64, 16, t, 0, 0, 0, None) == -9   # i must exceed k
    assert f(2, a, 200, 130, 200, 64, 16, t, 0, 0, 0, None) == -10  # j must exceed k
    assert f(0, a, 200, 130, 200, 64, 16, t, 0, 0, 3, None) == -11  # k beyond the tile grid
