"""The learned cost model's hand-written HIP kernels (forward, backward, Adam
training) against the FP64 CPU oracle of the same network: 5 -> 64 -> 64 ->
64 -> 1, ReLU, loss 1/(2n) sum (yhat - y)^2."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NP = 8769


def _data(n, seed, nmodels=1, scale=0.2):
    rng = np.random.default_rng(seed)
    p = (scale * rng.standard_normal((nmodels, NP))).astype(np.float32)
    X = rng.standard_normal((n, 5)).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    return p, X, y


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n,nmodels", [(1, 1), (257, 3), (5000, 5)])
def test_forward_matches_oracle(n, nmodels):
    import paper_1102_5328_amd as tq
    from paper_1102_5328_amd import _lib
    import torch
    p, X, _ = _data(n, 10 + n, nmodels)
    dp, dX = _dev(p), _dev(X)
    dy = torch.empty((nmodels, n), dtype=torch.float32, device="cuda")
    tq.check(_lib.lib().qr_mlp_forward(dp.data_ptr(), nmodels, dX.data_ptr(), n, dy.data_ptr(),
                                       None), "qr_mlp_forward")
    torch.cuda.synchronize()
    y = dy.cpu().numpy()
    for m in range(nmodels):
        ref = oracle.mlp_forward(p[m].astype(np.float64), X.astype(np.float64))
        # FP32 through three 64-wide layers: relative error ~1e-6, checked
        # against the scale of the outputs.
        err = np.max(np.abs(y[m] - ref)) / (np.max(np.abs(ref)) + 1e-30)
        assert err < 1e-4, (m, err)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4999])
def test_gradient_matches_oracle(n):
    """Hand-written backward (chunks of 64 rows, ragged tail) vs the oracle's
    analytic gradient in FP64: relative error <= 1e-5 in the 2-norm over all
    8769 entries, and the loss."""
    import paper_1102_5328_amd as tq
    from paper_1102_5328_amd import _lib
    import torch
    p, X, y = _data(n, 20 + n)
    dp, dX, dy = _dev(p[0]), _dev(X), _dev(y)
    g = torch.empty(NP, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    tq.check(_lib.lib().qr_mlp_grad(dp.data_ptr(), dX.data_ptr(), dy.data_ptr(), n, g.data_ptr(),
                                    loss.data_ptr(), None), "qr_mlp_grad")
    torch.cuda.synchronize()
    lo, go = oracle.mlp_grad(p[0].astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    gg = g.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    assert rel <= 1e-5, rel
    assert float(loss.cpu()) == pytest.approx(lo, rel=1e-5)


def test_training_reduces_loss_and_is_deterministic():
    """Adam on a smooth target: the full-batch loss (measured by the oracle)
    falls, and two runs from the same state and seed give the same bits."""
    import paper_1102_5328_amd as tq
    from paper_1102_5328_amd import _lib
    import torch
    rng = np.random.default_rng(5)
    n, nm = 2000, 4
    X = rng.standard_normal((n, 5)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 3]).astype(np.float32)
    p0 = (0.15 * rng.standard_normal((nm, NP))).astype(np.float32)
    before = [oracle.mlp_grad(p0[m].astype(np.float64), X.astype(np.float64),
                              y.astype(np.float64))[0] for m in range(nm)]
    outs = []
    for _ in range(2):
        dp = _dev(p0.copy())
        adam = torch.zeros(2 * nm * NP, dtype=torch.float32, device="cuda")
        lo = torch.empty(nm, dtype=torch.float32, device="cuda")
        dX, dy = _dev(X), _dev(y)
        tq.check(_lib.lib().qr_mlp_train(dp.data_ptr(), nm, adam.data_ptr(), dX.data_ptr(),
                                         dy.data_ptr(), n, 20, 64, 2e-3, 99, 0, lo.data_ptr(),
                                         None), "qr_mlp_train")
        torch.cuda.synchronize()
        outs.append(dp.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])
    for m in range(nm):
        after = oracle.mlp_grad(outs[0][m].astype(np.float64), X.astype(np.float64),
                                y.astype(np.float64))[0]
        assert after < 0.5 * before[m], (m, before[m], after)
