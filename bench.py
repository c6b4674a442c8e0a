"""Benchmark of the tile Householder QR on one MI355X.

A step is one full factorization of the N x N FP64 matrix (N = 16384,
entries N(0,1)) with the tuned (NB, IB): the input is restored from a
resident copy in HBM (device-to-device copy, inside the step) and then
factorized by qr_factor (one persistent launch). Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--n N] [--nb NB --ib IB]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (matrix and vector)
PEAK_HBM_TBPS = 8.0      # MI355X HBM3E
# Sources whose change invalidates recorded counters: the kernels and the
# host scheduler that orders their tasks.
KERNEL_SRC = [os.path.join(HERE, "paper_1102_5328_amd", "csrc", f)
              for f in ("tileqr_device.hip", "plan.cpp")]
TRAFFIC = os.path.join(HERE, "profiles", "traffic.txt")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(N, nb, ib, units):
    """HBM bytes per launch of the persistent kernel from the rocprofv3
    counter runs recorded in profiles/traffic.txt (FETCH_SIZE and WRITE_SIZE,
    each scaled by the same counter's reading for a device copy of known
    size), if they were taken on this kernel source and configuration; else
    None."""
    if not os.path.exists(TRAFFIC):
        return None
    h = kernel_source_hash()
    with open(TRAFFIC) as f:
        for line in f:
            w = dict(x.split("=", 1) for x in line.split() if "=" in x)
            if (w.get("kernel") == "tq_persistent" and w.get("src") == h and
                    int(w.get("N", -1)) == N and int(w.get("NB", -1)) == nb and
                    int(w.get("IB", -1)) == ib and int(w.get("units", 0)) == units):
                return float(w["bytes"])
    return None


def tuned_vs_exhaustive(N, nb, ib):
    """GFLOP/s of the chosen (NB, IB) as a percentage of the best of all
    39 pairs at this size, from the recorded config-2 sweep (None when the
    size was not swept)."""
    import json
    # the config-2 sweep taken with the current kernels; the tuner's own
    # database otherwise
    path = os.path.join(HERE, "paper_1102_5328_amd", "tuning", "sweep_timings.json")
    if not os.path.exists(path):
        path = os.path.join(HERE, "paper_1102_5328_amd", "tuning", "tune_timings.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        db = json.load(f)
    from paper_1102_5328_amd.tuner.runner import config2_pairs
    rates = {}
    for p in config2_pairs():
        r = db.get("normal:%d:%d:%d:%d:1" % (N, N, p[0], p[1]))
        if r is None:
            return None
        rates[p] = r["gflops"]
    if (nb, ib) not in rates:
        return None
    return round(100.0 * rates[(nb, ib)] / max(rates.values()), 2)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--nb", type=int, default=0)
    p.add_argument("--ib", type=int, default=0)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target duration of the CPU-oracle sample (0 = skip)")
    return p.parse_args()


def cpu_baseline(A_dev, target_s):
    """The oracle (unblocked FP64 Householder QR, OpenMP over trailing
    columns) timed on the first Householder steps of the same matrix."""
    import numpy as np
    import oracle
    M, N = A_dev.shape
    A = np.asfortranarray(A_dev.cpu().numpy())
    # Calibrate on a full-width copy (a narrow one runs the OpenMP update at a
    # lower rate and would overestimate the cost of a step): 8 steps.
    probe = A.copy(order="F")
    t0 = time.perf_counter()
    oracle.geqr2_steps_inplace(probe, 8)
    per_step = max((time.perf_counter() - t0) / 8.0, 1e-4)
    del probe
    steps = int(max(2, min(min(M, N), target_s / per_step)))
    t0 = time.perf_counter()
    oracle.geqr2_steps_inplace(A, steps)
    dt = time.perf_counter() - t0
    # Flops of steps 0..steps-1 of geqr2 (generation + rank-1 update).
    fl = 0.0
    for j in range(steps):
        fl += 3.0 * (M - j) + 4.0 * (M - j) * (N - j - 1)
    return {
        "value": round(fl / dt / 1e9, 3),
        "unit": "GFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "first %d of %d Householder steps of the same %dx%d N(0,1) matrix "
                  "(%.1f s)" % (steps, min(M, N), M, N, dt),
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the tile QR of one matrix runs on a single "
              "MI355X (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1102_5328_amd as tq
    from paper_1102_5328_amd import inputs

    N = args.n
    table = os.path.join(HERE, "paper_1102_5328_amd", "tuning", "decision_table.txt")
    if os.path.exists(table):
        tq.tune_load(table)
    nb, ib, src = args.nb, args.ib, 3
    if nb == 0 or ib == 0:
        tnb, tib, src = tq.tune(N, N, 1)
        nb, ib = nb or tnb, ib or tib
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A0 = inputs.torch_normal(N, N, seed=args.seed, device="cuda")
    A = tq.colmajor(N, N)
    T = torch.empty(tq.T_size(N, N, nb, ib), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        A.copy_(A0)
        if ev is not None:
            ev[0].record(stream)
        tq.factor(A, nb, ib, T)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
        tq.sync()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tq.sync()
    kern_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / args.steps
    units = tq.tune_units(N, N, 1)
    traffic = measured_traffic(N, nb, ib, units)
    # The ceiling of the FP64 matrix instruction itself at the kernel's
    # occupancy (two workgroups of four waves per CU), measured live by a
    # register-only probe, next to the published peak.
    ceil_tf, ceil_ghz = tq.mfma_probe(2, 50000)
    ms_per_step = dt * 1e3 / args.steps
    flops = tq.flops(N, N)
    value = flops / (ms_per_step * 1e-3) / 1e9
    achieved = flops / (kern_ms * 1e-3) / 1e12
    # Which roof bounds the path: its algorithmic intensity (metric flops over
    # the minimum HBM bytes: A read, R/V written, T written) against the
    # ridge point of the two peaks.
    alg_bytes = 16.0 * N * N + 8.0 * N * N * ib / nb
    intensity = flops / alg_bytes
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_TBPS * 1e12)
    bound = "mfma" if intensity >= ridge else "hbm"
    out = {
        "metric": "FP64 tile-QR GFLOP/s & % FP64 MFMA peak; tuned/predicted vs exhaustive-best %",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "tile Householder QR of one %dx%d FP64 N(0,1) matrix" % (N, N),
                   "M": N, "N": N, "NB": nb, "IB": ib, "tiling_source": src,
                   "compute_units": units or "all"},
        "pct_fp64_peak": round(100.0 * value / (PEAK_FP64_TFLOPS * 1e3), 2),
        "tuned_vs_exhaustive_pct": tuned_vs_exhaustive(N, nb, ib),
        "roofline": {"bound": bound, "achieved": round(achieved, 3),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                     "intensity_flop_per_byte": round(intensity, 1), "ridge": round(ridge, 2),
                     "algorithmic_bytes": alg_bytes,
                     "kernel": "tq_persistent (whole DAG, one launch)",
                     "kernel_ms": round(kern_ms, 3),
                     "hbm_GBps": (round(traffic / (kern_ms * 1e-3) / 1e9, 1)
                                  if traffic else None),
                     "mfma_probe_TFLOPs": round(ceil_tf, 2),
                     "frac_of_mfma_probe": round(achieved / ceil_tf, 4) if ceil_tf > 0 else None,
                     "probe_shader_GHz": round(ceil_ghz, 2)},
    }
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(A0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
