"""qr_set_compute_units with a stream masked to a subset of the compute
units (the analog of the paper's core count): the factorization sized for
32 units, on a stream restricted to them, still matches the oracle."""
import numpy as np
import pytest

import oracle
from paper_1102_5328_amd import inputs
from helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


def test_factor_on_cu_masked_stream():
    import torch
    import paper_1102_5328_amd as tq
    from paper_1102_5328_amd import experiments as E
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    A = inputs.uniform(700, 520, seed=11)
    dA = to_dev(A)
    tq.set_compute_units(32)
    hip, st = E._cu_masked_stream(32, ncu)
    try:
        stream = torch.cuda.ExternalStream(st.value)
        _, T, nb, ib = tq.factor(dA, 128, 32, stream=stream)
        tq.sync(stream)
    finally:
        tq.set_compute_units(0)
        torch.cuda.synchronize()
        hip.hipStreamDestroy(st)
    VR = to_host(dA)
    VRo, _ = oracle.geqr2(A)
    r = oracle.r_rel_diff(oracle.upper(VR), oracle.upper(VRo))
    assert r <= 1e-10 * np.linalg.cond(A), r
    with pytest.raises(tq.TileQRError):
        tq.set_compute_units(ncu + 1)


def test_tune_follows_the_callers_compute_units(tmp_path):
    """qr_tune answers from the table section tuned for the caller's unit
    count (Section 6.1's interpolation over cores): a caller limited to 64
    or 100 units gets the 64-unit entry, one without a setting or with the
    whole device the "all" entry, and the grid is the caller's."""
    import torch
    import paper_1102_5328_amd as tq
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    p = tmp_path / "budget.txt"
    p.write_text("entry 4000 4000 1 128 16 9.0\n"
                 "budget 64\n"
                 "entry 4000 4000 1 96 32 5.0 48\n")
    tq.tune_load(str(p))
    try:
        assert tq.tune(4000, 4000, 1)[:2] == (128, 16)
        tq.set_compute_units(64)
        assert tq.tune(4000, 4000, 1)[:2] == (96, 32)
        assert tq.tune_units(4000, 4000, 1) == 64
        tq.set_compute_units(100)
        assert tq.tune(4000, 4000, 1)[:2] == (96, 32)
        tq.set_compute_units(ncu)
        assert tq.tune(4000, 4000, 1)[:2] == (128, 16)
    finally:
        tq.set_compute_units(0)
        tq.tune_load(tq.SHIPPED_TABLE)
