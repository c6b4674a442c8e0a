"""Step 1 of the tuner (Section 5) on the GPU: the DSSRFB kernel benchmark
with warm tiles (No Flush) and with the caches flushed between calls. Both
must return a finite, positive time for every pair, and the flushed timing
cannot be faster than the warm one by more than the run-to-run noise."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nb,ib", [(64, 16), (128, 32)])
def test_step1_warm_and_flushed(nb, ib):
    import torch
    import paper_1102_5328_amd as tq
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    calls = 10
    warm = tq.ssrfb_bench(nb, ib, calls=calls)
    cold = tq.ssrfb_bench_flush(nb, ib, calls=calls, flush_bytes=256 << 20)
    flops = 4.0 * nb ** 3 * calls
    for t in (warm, cold):
        assert math.isfinite(t) and t > 0.0
    g_warm = flops * ncu / warm / 1e9   # one DSSRFB per workgroup per call
    g_cold = flops * ncu / cold / 1e9
    print(nb, ib, "warm %.0f GFLOP/s, flushed %.0f GFLOP/s" % (g_warm, g_cold))
    assert g_warm > 100.0 and g_cold > 10.0


def test_mfma_probe_rate_and_clock():
    """The FP64 MFMA probe: a finite, positive rate no higher than the
    published peak (78.6 TFLOP/s dense FP64), more waves per SIMD never much
    slower than one, and a shader clock within the chip's range."""
    import paper_1102_5328_amd as tq
    one, ghz1 = tq.mfma_probe(1, 20000)
    two, ghz2 = tq.mfma_probe(2, 20000)
    print("MFMA probe: 1 wave/SIMD %.2f TFLOP/s at %.2f GHz, 2 waves/SIMD %.2f TFLOP/s at %.2f GHz"
          % (one, ghz1, two, ghz2))
    for tf, ghz in ((one, ghz1), (two, ghz2)):
        assert math.isfinite(tf) and 1.0 < tf <= 78.6 * 1.02
        assert 0.5 < ghz < 3.0
    assert two > 0.9 * one
