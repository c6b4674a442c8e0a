"""End-to-end measurement flows on one GPU, each writing a JSON report:

  batched  2000 uneven matrices (M ~ U{64..1024}, N ~ U{32..M},
           uniform[-1, 1], seed 0), tiles per size class from qr_tune:
           one graph-captured persistent launch vs a loop of per-matrix
           launches (time ratio; results compared bit for bit).
  sweep    square N in {2048, 4096, 8192, 16384}, N(0, 1): GFLOP/s per
           (N, NB, IB) over the enabled grid (median of 6 after a warm-up).
  tune     the paper's pruned search (Step 1 -> heuristic -> Step 2 with and
           without pruning as you go) vs exhaustive search on tall, wide,
           square and ill-conditioned shapes; decision tables and tuning time.
  mlp      the learned cost model: timings -> training set, an ensemble of
           five 5-64-64-64-1 MLPs trained by the library's kernels, (NB, IB)
           predicted for 200 held-out shapes (M, N log-uniform in
           [256, 32768], seed 5), regret vs exhaustive search, fallback rate
           and gain over the decision table alone.

    python -m paper_1102_5328_amd.experiments {batched,sweep,tune} --out DIR [--db FILE]
    python -m paper_1102_5328_amd.experiments {collect-train,collect-heldout} --db FILE
                                              --out DIR [--budget SECONDS]
    python -m paper_1102_5328_amd.experiments mlp --db FILE --out DIR
    python -m paper_1102_5328_amd.experiments ship --out DIR   (DIR: a tune run's output)
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs
from .tuner import runner as R
from .tuner import step2 as S2

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING = os.path.join(HERE, "tuning")


def log(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ batched


def batched(out_dir, count=2000, seed=0, reps=5):
    import torch
    import paper_1102_5328_amd as tq
    table = os.path.join(TUNING, "decision_table.txt")
    if os.path.exists(table):
        tq.tune_load(table)
    shapes = inputs.batch_shapes(count, seed=seed)
    mats = inputs.batch_matrices(shapes, seed=seed)
    til = [tq.tune(m, n, count)[:2] for m, n in shapes]
    nbs, ibs = [t[0] for t in til], [t[1] for t in til]
    A0, As, Ts = [], [], []
    for (m, n), a, nb, ib in zip(shapes, mats, nbs, ibs):
        d = tq.colmajor(m, n)
        d.copy_(torch.from_numpy(np.ascontiguousarray(a.T)).t())
        A0.append(d)
        As.append(tq.colmajor(m, n))
        Ts.append(torch.empty(max(1, tq.T_size(m, n, nb, ib)), dtype=torch.float64, device="cuda"))
    flops = sum(tq.flops(m, n) for m, n in shapes)

    def restore():
        for a, a0 in zip(As, A0):
            a.copy_(a0)

    def timed(fn):
        ts = []
        for _ in range(reps + 1):
            restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn(As, nbs, ibs, Ts)
            tq.sync()
            ts.append(time.perf_counter() - t0)
        return ts[1:]

    t_loop = timed(tq.factor_loop)
    ref = [a.clone() for a in As]
    t_batch = timed(tq.factor_batched)
    same = all(torch.equal(a, r) for a, r in zip(As, ref))
    maxrel = max(float(torch.linalg.norm(a - r) / torch.linalg.norm(r)) for a, r in zip(As, ref))
    classes = {}
    for nb, ib in til:
        classes["%d,%d" % (nb, ib)] = classes.get("%d,%d" % (nb, ib), 0) + 1
    rep = {
        "count": count, "seed": seed, "flops": flops,
        "bytes": sum(8 * m * n for m, n in shapes),
        "tilings": classes,
        "loop_ms": [1e3 * t for t in t_loop], "batched_ms": [1e3 * t for t in t_batch],
        "loop_ms_median": 1e3 * float(np.median(t_loop)),
        "batched_ms_median": 1e3 * float(np.median(t_batch)),
        "speedup": float(np.median(t_loop) / np.median(t_batch)),
        "batched_gflops": flops / float(np.median(t_batch)) / 1e9,
        "loop_gflops": flops / float(np.median(t_loop)) / 1e9,
        "bitwise_equal": bool(same), "max_rel_diff_batched_vs_loop": maxrel,
        "timing": "host wall clock around the call and qr_sync, inputs restored before each "
                  "run (not timed); median of %d after one warm-up" % reps,
    }
    log("batched: loop %.2f ms, batched %.2f ms, speedup %.1fx, equal %s" %
        (rep["loop_ms_median"], rep["batched_ms_median"], rep["speedup"], same))
    with open(os.path.join(out_dir, "batched_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return rep


def _pow2_class(x):
    c = 1
    while c < x:
        c *= 2
    return c


def batched_tune(out_dir, db, count=2000, seed=0, reps=3):
    """Step 2 for the batch. The matrices are grouped in size classes (M and
    N rounded up to powers of two); for each class, every enabled (NB, IB) is
    timed on a batched launch of the class's matrices. One launch runs every
    matrix in the register class of its largest tile order, so per-class
    choices are then combined within each register class (NB <= 64, NB <= 128)
    and, with every uniform pair, timed on the whole batch; the fastest
    whole-batch assignment gives the decision-table entries (class M, class
    N, batch count). Returns the entries."""
    import torch
    import paper_1102_5328_amd as tq
    shapes = inputs.batch_shapes(count, seed=seed)
    mats = inputs.batch_matrices(shapes, seed=seed)
    classes = {}
    for b, (m, n) in enumerate(shapes):
        classes.setdefault((_pow2_class(m), _pow2_class(n)), []).append(b)
    meas = R.Measurer(db)
    pairs = R.config2_pairs()
    entries = {}
    per_class = {}
    t0 = time.perf_counter()
    for (cm, cn), idx in sorted(classes.items()):
        A0 = []
        for b in idx:
            d = tq.colmajor(*shapes[b])
            d.copy_(torch.from_numpy(np.ascontiguousarray(mats[b].T)).t())
            A0.append(d)
        As = [tq.colmajor(*shapes[b]) for b in idx]
        fl = sum(tq.flops(*shapes[b]) for b in idx)
        res = {}
        for nb, ib in pairs:
            key = "batched:%d:%d:%d:%d:%d" % (cm, cn, nb, ib, count)
            if key not in meas.db:
                Ts = [torch.empty(max(1, tq.T_size(*shapes[b], nb, ib)), dtype=torch.float64,
                                  device="cuda") for b in idx]
                nbs, ibs = [nb] * len(idx), [ib] * len(idx)
                ts = []
                for r in range(reps + 1):
                    for a, a0 in zip(As, A0):
                        a.copy_(a0)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    tq.factor_batched(As, nbs, ibs, Ts)
                    tq.sync()
                    ts.append(time.perf_counter() - t1)
                g = [fl / t / 1e9 for t in ts[1:]]
                gm = float(np.median(g))
                # M, N of the record: the class's geometric-mean shape.
                mg = int(round(math.exp(np.mean([math.log(shapes[b][0]) for b in idx]))))
                ng = int(round(math.exp(np.mean([math.log(shapes[b][1]) for b in idx]))))
                meas.db[key] = {"gflops": gm, "max": max(g), "runs": g, "seconds": sum(ts),
                                "M": mg, "N": ng, "nb": nb, "ib": ib, "batch": count,
                                "kind": "batched", "class": [cm, cn], "matrices": len(idx)}
            res[(nb, ib)] = meas.db[key]["gflops"]
        per_class[(cm, cn)] = res
        best = max(res, key=lambda p: (res[p], -p[0]))
        log("batch class %dx%d (%d matrices): best %s %.1f GFLOP/s (%.0f s)" %
            (cm, cn, len(idx), best, res[best], time.perf_counter() - t0))
        meas.save()
    # Whole-batch assignments: per-class best within each register class,
    # and every uniform pair.
    groups = {"nb<=64": [p for p in pairs if p[0] <= 64], "nb<=128": [p for p in pairs if p[0] > 64]}
    cands = {}
    for gname, gp in groups.items():
        cands["per-class " + gname] = {c: max(gp, key=lambda p: (per_class[c][p], -p[0]))
                                       for c in classes}
    for p in pairs:
        cands["uniform %d/%d" % p] = {c: p for c in classes}
    A0 = []
    for b in range(count):
        d = tq.colmajor(*shapes[b])
        d.copy_(torch.from_numpy(np.ascontiguousarray(mats[b].T)).t())
        A0.append(d)
    As = [tq.colmajor(*shapes[b]) for b in range(count)]
    fl_all = sum(tq.flops(*sh) for sh in shapes)
    whole = {}
    for name, assign in cands.items():
        til = [assign[(_pow2_class(m), _pow2_class(n))] for m, n in shapes]
        Ts = [torch.empty(max(1, tq.T_size(*shapes[b], *til[b])), dtype=torch.float64,
                          device="cuda") for b in range(count)]
        nbs, ibs = [t[0] for t in til], [t[1] for t in til]
        ts = []
        for r in range(reps + 1):
            for a, a0 in zip(As, A0):
                a.copy_(a0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tq.factor_batched(As, nbs, ibs, Ts)
            tq.sync()
            ts.append(time.perf_counter() - t1)
        whole[name] = fl_all / float(np.median(ts[1:])) / 1e9
        log("whole batch, %s: %.1f GFLOP/s" % (name, whole[name]))
        del Ts
    pick = max(whole, key=whole.get)
    log("whole batch: %s is fastest" % pick)
    for (cm, cn), idx in classes.items():
        nb, ib = cands[pick][(cm, cn)]
        rec = meas.db["batched:%d:%d:%d:%d:%d" % (cm, cn, nb, ib, count)]
        entries[(rec["M"], rec["N"])] = (nb, ib, per_class[(cm, cn)][(nb, ib)])
    with open(os.path.join(out_dir, "batched_tune.json"), "w") as f:
        json.dump({"%dx%d" % k: list(v) for k, v in entries.items()}, f, indent=1)
    with open(os.path.join(out_dir, "batched_tune_whole.json"), "w") as f:
        json.dump({"whole_batch_gflops": whole, "chosen": pick}, f, indent=1)
    return entries


# ------------------------------------------------------------- sweep / tune


def sweep(out_dir, db):
    m = R.Measurer(db, reps=6)
    s1, t1 = R.step1_gpu(R.config2_pairs())
    log("step1 (%.1f s): %s" % (t1, {"%d,%d" % p: round(v, 1) for p, v in s1.items()}))
    res = R.sweep_square(m, log=log)
    m.save()
    with open(os.path.join(out_dir, "sweep_report.json"), "w") as f:
        json.dump({"step1_gflops": {"%d,%d" % p: v for p, v in s1.items()}, "step1_seconds": t1,
                   "sweep": res}, f, indent=1)
    return res


def tune(out_dir, db):
    m = R.Measurer(db, reps=6)
    rep = R.tune_search(m, out_dir, log=log)
    m.save()
    return rep


def _read_entries(path):
    """Entries of a decision table file: (M, N, batch, NB, IB, gflops, units, p)."""
    out = []
    with open(path) as f:
        for line in f:
            w = line.split()
            if w and w[0] == "entry":
                out.append(tuple(int(x) for x in w[1:6]) + (float(w[6]),) +
                           ((int(w[7]),) if len(w) > 7 else (0,)) +
                           ((int(w[8]),) if len(w) > 8 else (1,)))
    return out


def _write_entry(f, e):
    M, N, b, nb, ib, g, u, p = e
    if p > 1:
        f.write("entry %d %d %d %d %d %.3f %d %d\n" % (M, N, b, nb, ib, g, u, p))
    elif u:
        f.write("entry %d %d %d %d %d %.3f %d\n" % (M, N, b, nb, ib, g, u))
    else:
        f.write("entry %d %d %d %d %d %.3f\n" % (M, N, b, nb, ib, g))


def ship_table(tune_dir, out_path, heuristic="2r", batch_count=2000, src_name=None):
    """The decision table the library ships: the Step-2 decisions for single
    matrices (`src_name` in tune_dir, by default heuristic's PSPAYG table;
    entries may carry a unit count and a row-domain count) plus the
    per-size-class decisions of the batched tuning (entries with the batch
    count), then one section per compute-unit budget tuned by tune-budgets
    (decision_table_budget_C.txt)."""
    src = os.path.join(tune_dir, src_name or "decision_table_h%s_pspayg.txt" % heuristic)
    entries = _read_entries(src)
    default = (128, 16)
    bt = os.path.join(tune_dir, "batched_tune.json")
    if os.path.exists(bt):
        with open(bt) as f:
            for k, (nb, ib, g) in json.load(f).items():
                m, n = (int(x) for x in k.split("x"))
                entries.append((m, n, batch_count, nb, ib, g, 0, 1))
    big = max((e for e in entries if e[2] == 1), key=lambda e: e[0] * e[1], default=None)
    if big is not None:
        default = (big[3], big[4])
    budgets = []
    for name in sorted(os.listdir(tune_dir)):
        if name.startswith("decision_table_budget_") and name.endswith(".txt"):
            c = int(name[len("decision_table_budget_"):-4])
            budgets.append((c, _read_entries(os.path.join(tune_dir, name))))
    budgets.sort()
    with open(out_path, "w") as f:
        f.write("# tileqr decision table: entry M N batch NB IB gflops [units [p]]\n")
        f.write("# single matrices: Step 2 over the pairs of heuristic %s (%s), each pair at\n"
                "# its best row-domain count p;\n" % (heuristic, os.path.basename(src)))
        f.write("# batch %d: per size class (M, N rounded up to powers of two; the entry holds\n"
                "# the class's geometric-mean shape)\n" % batch_count)
        f.write("default %d %d\n" % default)
        for e in sorted(entries, key=lambda e: (e[2], e[0], e[1])):
            _write_entry(f, e)
        for c, ents in budgets:
            f.write("# callers limited to %d compute units (qr_set_compute_units)\n" % c)
            f.write("budget %d\n" % c)
            for e in sorted(ents, key=lambda e: (e[2], e[0], e[1])):
                _write_entry(f, e)
    return entries


def step1_cold(out_dir, db, flush_bytes=1 << 30):
    """Step 1 with warm and with cold caches, and what each pre-selects: the
    Step-2 analysis of every heuristic is replayed from the recorded runs
    (the database must hold every pair on the grid and the test shapes)."""
    pairs = R.config2_pairs()
    warm, t_warm = R.step1_gpu(pairs)
    cold, t_cold = R.step1_gpu(pairs, flush_bytes=flush_bytes)
    log("step1 warm (%.1f s): %s" % (t_warm, {"%d,%d" % p: round(v) for p, v in warm.items()}))
    log("step1 cold (%.1f s): %s" % (t_cold, {"%d,%d" % p: round(v) for p, v in cold.items()}))
    rep = {"flush_bytes": flush_bytes,
           "step1_warm": {"%d,%d" % p: v for p, v in warm.items()}, "step1_warm_seconds": t_warm,
           "step1_cold": {"%d,%d" % p: v for p, v in cold.items()}, "step1_cold_seconds": t_cold}
    for name, s1, t1 in (("warm", warm, t_warm), ("cold", cold, t_cold)):
        sub = os.path.join(out_dir, "step1_" + name)
        os.makedirs(sub, exist_ok=True)
        m = R.Measurer(db, offline=True, verbose=False)
        r = R.tune_search(m, sub, step1=(s1, t1), log=log)
        rep[name] = {h: {"preselected": e["preselected"],
                         "PSPAYG_avg_pct_of_ES": e["PSPAYG"]["avg_pct_of_ES"],
                         "PSPAYG_optimum": e["PSPAYG"]["optimum"],
                         "PSPAYG_seconds": r["tuning_seconds"]["H%s_PSPAYG" % h]}
                     for h, e in r["heuristics"].items()}
    with open(os.path.join(out_dir, "step1_cold_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return rep


def _cu_masked_stream(cus, ncu):
    """A stream restricted to the first `cus` compute units
    (hipExtStreamCreateWithCUMask of the HIP runtime torch loaded)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    words = (ncu + 31) // 32
    mask = (ctypes.c_uint32 * words)()
    for c in range(cus):
        mask[c // 32] |= 1 << (c % 32)
    st = ctypes.c_void_p()
    rc = hip.hipExtStreamCreateWithCUMask(ctypes.byref(st), ctypes.c_uint32(words), mask)
    if rc != 0:
        raise RuntimeError("hipExtStreamCreateWithCUMask failed: %d" % rc)
    return hip, st


def cu_scaling(out_dir, sizes=(4096, 8192, 16384), cus_list=(32, 64, 128, 256),
               pairs=((64, 16), (96, 16), (128, 16), (128, 32)), reps=3):
    """Strong scaling over compute units, the analog of the paper's core
    count: the factorization on a stream masked to `cus` units, with the
    grid and schedule sized for them, for a few (NB, IB) per size."""
    import torch
    import paper_1102_5328_amd as tq
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    try:
        for cus in cus_list:
            tq.set_compute_units(cus)
            hip, st = _cu_masked_stream(cus, ncu)
            stream = torch.cuda.ExternalStream(st.value)
            for N in sizes:
                A0 = inputs.torch_normal(N, N, seed=0)
                A = tq.colmajor(N, N)
                res = {}
                for nb, ib in pairs:
                    T = torch.empty(tq.T_size(N, N, nb, ib), dtype=torch.float64, device="cuda")
                    ts = []
                    for r in range(reps + 1):
                        A.copy_(A0)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        tq.factor(A, nb, ib, T, stream=stream)
                        tq.sync(stream)
                        ts.append(time.perf_counter() - t0)
                    g = tq.flops(N, N) / float(np.median(ts[1:])) / 1e9
                    res["%d,%d" % (nb, ib)] = g
                    log("cus=%d N=%d nb=%d ib=%d: %.1f GFLOP/s" % (cus, N, nb, ib, g))
                    del T
                out.setdefault(str(cus), {})[str(N)] = res
                del A, A0
            torch.cuda.synchronize()
            hip.hipStreamDestroy(st)
    finally:
        tq.set_compute_units(0)
    summary = {}
    for N in sizes:
        row = {}
        for cus in cus_list:
            r = out[str(cus)][str(N)]
            best = max(r, key=r.get)
            row[str(cus)] = {"best": best, "gflops": r[best]}
        base = row[str(cus_list[0])]["gflops"]
        for cus in cus_list:
            row[str(cus)]["speedup_vs_%d" % cus_list[0]] = row[str(cus)]["gflops"] / base
            row[str(cus)]["efficiency"] = (row[str(cus)]["gflops"] / base) / (cus / cus_list[0])
        summary[str(N)] = row
    rep = {"cus": list(cus_list), "sizes": list(sizes), "pairs": [list(p) for p in pairs],
           "gflops": out, "summary": summary,
           "mask": "the first `cus` bits of the compute-unit mask"}
    with open(os.path.join(out_dir, "cu_scaling_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return rep


def tune_units(out_dir, db, units_list=(64, 128, 0)):
    """Step 2 with the compute-unit count as a third tunable: every
    pre-selected pair of the shipped heuristic at each unit count (0: all)
    on the size grid; the best (NB, IB, units) per grid shape makes the
    table, which is then scored on the test shapes against the exhaustive
    search over the pairs on the whole device."""
    import paper_1102_5328_amd as tq
    ps = shipped_preselection()
    meas = R.Measurer(db)
    dec, t = {}, 0.0
    for (M, N) in R.STEP2_GRID:
        best = None
        for nb, ib in ps:
            for u in units_list:
                g, sec = meas.measure(M, N, nb, ib, units=u)
                t += sec
                if best is None or g > best[2]:
                    best = (nb, ib, g, u)
        dec[(M, N)] = best
        meas.save()
        log("grid %dx%d: best NB=%d IB=%d units=%s %.1f GFLOP/s" %
            (M, N, best[0], best[1], best[3] or "all", best[2]))
    path = os.path.join(out_dir, "decision_table_h2r_units.txt")
    S2.write_table(path, dec, comment="heuristic 2r pairs x compute units %s (0: all)" %
                   (list(units_list),))
    tq.tune_load(path)
    rows = []
    for kind, M, N in R.TEST_SHAPES:
        nb, ib, _ = tq.tune(M, N, 1)
        u = tq.tune_units(M, N, 1)
        g = meas.measure(M, N, nb, ib, kind=kind, units=u)[0]
        es = max(meas.db[R.Measurer.key(kind, M, N, p[0], p[1])]["gflops"]
                 for p in R.config2_pairs())
        rows.append({"kind": kind, "M": M, "N": N, "nb": nb, "ib": ib, "units": u,
                     "gflops": g, "es_pairs_gflops": es, "pct_of_es_pairs": S2.percent(g, es)})
        log("test %s %dx%d: NB=%d IB=%d units=%s %.1f GFLOP/s = %.1f%% of the pairs-only ES" %
            (kind, M, N, nb, ib, u or "all", g, 100.0 * g / es))
    meas.save()
    rep = {"units": list(units_list), "preselected": [list(p) for p in ps],
           "step2_seconds": t, "grid": {"%dx%d" % k: list(v) for k, v in dec.items()},
           "test": rows, "avg_pct_of_es_pairs": round(float(np.mean([r["pct_of_es_pairs"]
                                                                    for r in rows])), 2)}
    with open(os.path.join(out_dir, "tune_units_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return rep


BUDGET_GRID = [(1024, 1024), (2048, 2048), (4096, 4096), (8192, 8192),
               (16384, 256), (65536, 256), (4096, 1024), (16384, 1024)]


def tune_budgets(out_dir, db, budgets=(32, 64, 128)):
    """The (size, compute units) decision of Section 6.1 (the paper
    interpolates over the core count): for each budget C, Step 2 (PSPAYG) of
    the shipped heuristic's pre-selected pairs, each at its best row-domain
    count, on a stream restricted to C compute units with the grid sized for
    them; the decisions go to decision_table_budget_C.txt, a section that
    qr_tune consults for callers limited to C units."""
    import torch
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    ps = shipped_preselection()
    meas = R.Measurer(db, reps=4)
    rep = {"preselected": [list(p) for p in ps], "grid": ["%dx%d" % s for s in BUDGET_GRID]}
    for c in budgets:
        hip, st = _cu_masked_stream(c, ncu)
        meas.masked = (c, torch.cuda.ExternalStream(st.value))
        try:
            m = lambda M, N, nb, ib: meas.measure_best_p(M, N, nb, ib, units=c)[:2]
            table, t = S2.step2(BUDGET_GRID, ps, m, payg=True)
            dec = {}
            for s_, d in S2.decisions(table).items():
                p = meas.measure_best_p(s_[0], s_[1], d[0], d[1], units=c)[2]
                dec[s_] = (d[0], d[1], d[2], c, p)
        finally:
            meas.masked = None
            torch.cuda.synchronize()
            hip.hipStreamDestroy(st)
        meas.save()
        S2.write_table(os.path.join(out_dir, "decision_table_budget_%d.txt" % c), dec,
                       comment="heuristic 2r pairs, PSPAYG, %d compute units (masked stream)" % c)
        rep[str(c)] = {"step2_seconds": t,
                       "decisions": {"%dx%d" % k: list(v) for k, v in dec.items()}}
        log("budget %d: step2 %.1f s, %s" % (c, t, {"%dx%d" % k: v[:2] + v[4:] for k, v in dec.items()}))
    with open(os.path.join(out_dir, "tune_budgets_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return rep


# -------------------------------------------------------------------- MLP

NP = 8769


def features(M, N, nb, ib, batch):
    return [math.log(M), math.log(N), math.log(nb), ib / float(nb), math.log(batch)]


def _training_rows(db):
    X, y = [], []
    for r in db.values():
        if r.get("kind", "normal") not in ("normal", "batched") or r["gflops"] <= 0:
            continue
        if r.get("p", 1) > 1 or r.get("units", 0):  # the model's regime: flat tree, whole device
            continue
        X.append(features(r["M"], r["N"], r["nb"], r["ib"], r.get("batch", 1)))
        y.append(math.log(r["gflops"]))
    return np.array(X, dtype=np.float64), np.array(y, dtype=np.float64)


def _init_params(seed):
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NP, dtype=np.float32)

    def fill(off, fan_out, fan_in):
        lim = math.sqrt(6.0 / fan_in)
        p[off:off + fan_out * fan_in] = rng.uniform(-lim, lim, size=fan_out * fan_in)
    fill(0, 64, 5)
    fill(384, 64, 64)
    fill(4544, 64, 64)
    fill(8704, 1, 64)
    return p


def train_ensemble(X, y, nmodels=5, epochs=300, batch=64, lr=1e-3, seed=0):
    """Standardises features and targets and trains `nmodels` models at once
    with the library's kernels. Returns (params, fmean, fstd, ymean, ystd,
    final losses, seconds)."""
    import torch
    import paper_1102_5328_amd as tq
    from . import _lib
    fmean, fstd = X.mean(0), X.std(0)
    fstd[fstd == 0] = 1.0
    ymean, ystd = float(y.mean()), float(y.std() or 1.0)
    Xs = ((X - fmean) / fstd).astype(np.float32)
    ys = ((y - ymean) / ystd).astype(np.float32)
    p0 = np.stack([_init_params(seed + m) for m in range(nmodels)])
    dp = torch.from_numpy(p0).cuda()
    adam = torch.zeros(2 * nmodels * NP, dtype=torch.float32, device="cuda")
    dX = torch.from_numpy(np.ascontiguousarray(Xs)).cuda()
    dy = torch.from_numpy(ys).cuda()
    lo = torch.empty(nmodels, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    step = 0
    chunk = 25
    steps_per_epoch = (len(ys) + batch - 1) // batch
    for e0 in range(0, epochs, chunk):
        ne = min(chunk, epochs - e0)
        tq.check(_lib.lib().qr_mlp_train(dp.data_ptr(), nmodels, adam.data_ptr(), dX.data_ptr(),
                                         dy.data_ptr(), len(ys), ne, batch, lr, seed, step,
                                         lo.data_ptr(), None), "qr_mlp_train")
        torch.cuda.synchronize()
        step += ne * steps_per_epoch
        log("  mlp epochs %d: loss %s" % (e0 + ne, np.round(lo.cpu().numpy(), 4).tolist()))
    sec = time.perf_counter() - t0
    return (dp.cpu().numpy(), fmean, fstd, ymean, ystd, lo.cpu().numpy().tolist(), sec)


TRAIN_SHAPES = dict(count=420, seed=11, lo=256, hi=16384)
# Candidates of the cost model: the tile orders up to 256 with IB of 16, 32
# or 64 dividing them (every size's best pair in the square sweep is among
# them; the larger tiles and IBs trail at every size).
MLP_PAIRS = [(nb, ib) for nb in (64, 96, 128, 192, 256) for ib in (16, 32, 64) if nb % ib == 0]
TEST_SHAPES = dict(count=200, seed=5)


def _shape_sets():
    test_shapes = inputs.log_uniform_shapes(TEST_SHAPES["count"], seed=TEST_SHAPES["seed"])
    tset = set(test_shapes)
    train = inputs.log_uniform_shapes(TRAIN_SHAPES["count"], seed=TRAIN_SHAPES["seed"],
                                      lo=TRAIN_SHAPES["lo"], hi=TRAIN_SHAPES["hi"])
    return [s for s in train if s not in tset], test_shapes


def collect(db, which, budget_s, reps=2):
    """Measures every enabled (NB, IB) pair on the training shapes (kind
    'normal') or on the held-out shapes (kind 'heldout': never used for
    training) until done or `budget_s` seconds have passed; resumable, the
    database keeps what was measured. Returns True when complete."""
    pairs = MLP_PAIRS
    meas = R.Measurer(db, reps=reps)
    train, test = _shape_sets()
    shapes, kind = (train, "normal") if which == "train" else (test, "heldout")
    t0 = time.perf_counter()
    done = True
    for q, (M, N) in enumerate(shapes):
        if time.perf_counter() - t0 > budget_s:
            done = False
            break
        for nb, ib in pairs:
            meas.measure(M, N, nb, ib, kind=kind)
        if q % 5 == 0:
            meas.save()
        log("%s shape %d/%d %dx%d (%.0f s)" % (which, q + 1, len(shapes), M, N,
                                                time.perf_counter() - t0))
    meas.save()
    return done


def heldout_es(db):
    """{(M, N): {pair: median GFLOP/s}} of the exhaustive search on the
    held-out shapes (every pair must have been measured)."""
    pairs = MLP_PAIRS
    _, test_shapes = _shape_sets()
    return {(M, N): {p: db[R.Measurer.key("heldout", M, N, p[0], p[1])]["gflops"] for p in pairs}
            for (M, N) in test_shapes}


def shipped_preselection():
    """The pre-selected pairs of the shipped heuristic (the GPU variant when
    the tuning report has it), the fallback search's candidates."""
    rep_path = os.path.join(TUNING, "tuning_report.json")
    if os.path.exists(rep_path):
        with open(rep_path) as f:
            heur = json.load(f)["heuristics"]
        return [tuple(p) for p in heur.get("2r", heur.get("2"))["preselected"]]
    return R.config2_pairs()


def ensemble_predict(model, M, N, batch=1, pairs=None):
    """Predicted GFLOP/s of every candidate pair for one shape by every
    member of the ensemble (qr_mlp_forward on the device): nmodels x ncand."""
    import torch
    import paper_1102_5328_amd as tq
    from . import _lib
    params, fmean, fstd, ymean, ystd = model
    pairs = pairs or MLP_PAIRS
    X = np.array([features(M, N, nb, ib, batch) for nb, ib in pairs])
    Xs = torch.from_numpy(((X - fmean) / fstd).astype(np.float32)).cuda()
    P = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
    y = torch.empty((len(params), len(pairs)), dtype=torch.float32, device="cuda")
    tq.check(_lib.lib().qr_mlp_forward(P.data_ptr(), len(params), Xs.data_ptr(), len(pairs),
                                       y.data_ptr(), None), "qr_mlp_forward")
    torch.cuda.synchronize()
    return np.exp(y.cpu().numpy().astype(np.float64) * ystd + ymean)


def evaluate(es, model, table=None, ps=None):
    """Regret on the held-out shapes of three ways of choosing (NB, IB):
    qr_tune with the model installed (its choice, or the pruned search on the
    shape, i.e. the best pre-selected pair, when it reports a spread above
    5 %), the model alone (the ensemble-mean best), and the decision table
    alone. model = (params, fmean, fstd, ymean, ystd). Also reports how often
    the other reading of the spread, (max - min) / mean of the predicted
    GFLOP/s at the chosen pair, would have fallen back."""
    import paper_1102_5328_amd as tq
    pairs = MLP_PAIRS
    cand = np.array(pairs, dtype=np.int32).reshape(-1)
    params, fmean, fstd, ymean, ystd = model
    table = table or os.path.join(TUNING, "decision_table.txt")
    tq.tune_load(table if os.path.exists(table) else os.devnull)
    ps = [p for p in (ps or shipped_preselection()) if p in pairs] or pairs
    rows = []
    t_choose = 0.0
    skipped = 0
    try:
        for (M, N), rates in es.items():
            # the model and the timings are of the flat tree: shapes whose
            # table entry is a tree (tall shapes) are answered by the table
            # alone and are not scored here
            if tq.tune_domains(M, N, 1) > 1:
                skipped += 1
                continue
            tq.check(_lib_set_model(None, 0, fmean, fstd, ymean, ystd, cand), "model off")
            tnb, tib, _ = tq.tune(M, N, 1)
            tq.check(_lib_set_model(params, len(params), fmean, fstd, ymean, ystd, cand), "model on")
            t0 = time.perf_counter()
            qnb, qib, src = tq.tune(M, N, 1)
            t_choose += time.perf_counter() - t0
            g = ensemble_predict(model, M, N, 1, pairs)
            c = int(np.argmax(g.mean(0)))
            own = pairs[c]
            spread_range = float((g[:, c].max() - g[:, c].min()) / g[:, c].mean())
            spread_loss = float(max(1.0 - g[k, c] / g[k].max() for k in range(len(g))))
            best = max(rates, key=rates.get)
            fallback = bool(src & 8)
            if not fallback:
                assert (qnb, qib) == own, ((M, N), (qnb, qib), own)
            choice = max(ps, key=lambda p: rates[p]) if fallback else own
            rows.append({"M": M, "N": N, "best": list(best), "best_gflops": rates[best],
                         "model": list(own), "model_gflops": rates[own],
                         "spread": spread_loss, "spread_range": spread_range,
                         "fallback": fallback, "chosen": list(choice),
                         "chosen_gflops": rates[choice], "table": [tnb, tib],
                         "table_gflops": rates.get((tnb, tib), float("nan"))})
    finally:
        _lib_set_model(None, 0, fmean, fstd, ymean, ystd, cand)
    reg = np.array([1.0 - r["chosen_gflops"] / r["best_gflops"] for r in rows])
    reg_t = np.array([1.0 - r["table_gflops"] / r["best_gflops"] for r in rows])
    reg_m = np.array([1.0 - r["model_gflops"] / r["best_gflops"] for r in rows])
    fl = np.array([tq.flops(r["M"], r["N"]) for r in rows])
    return {
        "n_test": len(rows), "n_tree_shapes_skipped": skipped,
        "fallback_rate": float(np.mean([r["fallback"] for r in rows])),
        "fallback_rate_range_reading": float(np.mean([r["spread_range"] > 0.05 for r in rows])),
        "preselected_fallback_pairs": [list(p) for p in ps],
        "regret_mean": float(reg.mean()), "regret_max": float(reg.max()),
        "regret_model_only_mean": float(reg_m.mean()), "regret_model_only_max": float(reg_m.max()),
        "regret_table_only_mean": float(np.nanmean(reg_t)),
        "regret_table_only_max": float(np.nanmax(reg_t)),
        "within_3pct": float(np.mean(reg <= 0.03)),
        "within_3pct_model_only": float(np.mean(reg_m <= 0.03)),
        "within_3pct_table_only": float(np.mean(reg_t <= 0.03)),
        "flops_weighted_regret": float(np.sum(reg * fl) / np.sum(fl)),
        "flops_weighted_regret_model_only": float(np.sum(reg_m * fl) / np.sum(fl)),
        "flops_weighted_regret_table_only": float(np.nansum(reg_t * fl) / np.sum(fl)),
        "choose_ms_mean": 1e3 * t_choose / max(1, len(rows)),
        "rows": rows,
    }


def mlp(out_dir, db):
    """Trains the ensemble on the database's timings and evaluates it on the
    held-out shapes (which must all have been measured)."""
    meas = R.Measurer(db)
    es = heldout_es(meas.db)
    X, y = _training_rows(meas.db)
    log("training rows: %d" % len(y))
    params, fmean, fstd, ymean, ystd, losses, t_train = train_ensemble(X, y)
    rep = {"train_rows": int(len(y)), "train_seconds": t_train, "final_losses": losses,
           "pairs": [list(p) for p in MLP_PAIRS]}
    rep.update(evaluate(es, (params, fmean, fstd, ymean, ystd)))
    log("mlp: regret mean %.4f max %.4f (model only %.4f, table only %.4f), fallback %.2f" %
        (rep["regret_mean"], rep["regret_max"], rep["regret_model_only_mean"],
         rep["regret_table_only_mean"], rep["fallback_rate"]))
    with open(os.path.join(out_dir, "mlp_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    with open(os.path.join(out_dir, "mlp_model.json"), "w") as f:
        json.dump({"params": params.tolist(), "fmean": fmean.tolist(), "fstd": fstd.tolist(),
                   "ymean": ymean, "ystd": ystd,
                   "cand": np.array(MLP_PAIRS).reshape(-1).tolist()}, f)
    return rep


def _lib_set_model(params, nmodels, fmean, fstd, ymean, ystd, cand):
    import ctypes
    from . import _lib
    F = ctypes.POINTER(ctypes.c_float)
    fm = np.ascontiguousarray(fmean, dtype=np.float32)
    fs = np.ascontiguousarray(fstd, dtype=np.float32)
    c = np.ascontiguousarray(cand, dtype=np.int32)
    if nmodels == 0:
        return _lib.lib().qr_tune_set_model(None, 0, None, None, 0.0, 1.0, None, 0)
    p = np.ascontiguousarray(params, dtype=np.float32)
    return _lib.lib().qr_tune_set_model(p.ctypes.data_as(F), nmodels, fm.ctypes.data_as(F),
                                        fs.ctypes.data_as(F), ymean, ystd,
                                        c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(c) // 2)


def mfma_ceiling(out_dir):
    """The FP64 MFMA probe at 1..4 waves per SIMD, next to the Step-1 DSSRFB
    rate (128/16) at one and two workgroups per compute unit: how close the
    update kernel runs to what the matrix instruction itself sustains."""
    import torch
    import paper_1102_5328_amd as tq
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    rows = []
    for w in (1, 2, 3, 4):
        tf, ghz = tq.mfma_probe(w, 50000)
        rows.append({"waves_per_simd": w, "probe_TFLOPs": tf, "shader_GHz": ghz})
        log("probe: %d wave(s)/SIMD %.2f TFLOP/s at %.2f GHz (%.1f %% of 78.6)" %
            (w, tf, ghz, 100.0 * tf / 78.6))
    step1 = []
    for wpc in (1, 2):
        calls = 50
        sec = tq.ssrfb_bench(128, 16, calls, wpc * ncu)
        tf = 4.0 * 128 ** 3 * calls * wpc * ncu / sec / 1e12
        ref = rows[wpc - 1]["probe_TFLOPs"]
        step1.append({"workgroups_per_cu": wpc, "TFLOPs": tf, "frac_of_probe": tf / ref})
        log("Step 1 DSSRFB 128/16: %d workgroup(s)/CU %.2f TFLOP/s = %.3f of the probe" %
            (wpc, tf, tf / ref))
    with open(os.path.join(out_dir, "mfma_ceiling_report.json"), "w") as f:
        json.dump({"probe": rows, "step1_128_16": step1}, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["batched", "batched-tune", "sweep", "tune", "step1-cold",
                                     "cu-scaling", "tune-units", "tune-budgets", "ship",
                                     "collect-train",
                                     "collect-heldout", "mlp", "mfma-ceiling"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--db", default=None, help="JSON measurement database (read and extended)")
    ap.add_argument("--budget", type=float, default=600.0, help="seconds of measuring (collect)")
    ap.add_argument("--src", default=None, help="ship: the single-matrix decision table in --out")
    ap.add_argument("--units", default="64,128,0",
                    help="tune-units: compute-unit counts to try (0: all)")
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    if a.what == "ship":
        ship_table(a.out, os.path.join(TUNING, "decision_table.txt"), src_name=a.src)
        return 0
    import torch
    torch.cuda.set_device(0)
    db = a.db or os.path.join(a.out, "measurements.json")
    if a.what == "batched":
        batched(a.out)
    elif a.what == "batched-tune":
        batched_tune(a.out, db)
    elif a.what == "sweep":
        sweep(a.out, db)
    elif a.what == "tune":
        tune(a.out, db)
    elif a.what == "step1-cold":
        step1_cold(a.out, db)
    elif a.what == "cu-scaling":
        cu_scaling(a.out)
    elif a.what == "tune-units":
        tune_units(a.out, db, tuple(int(x) for x in a.units.split(",")))
    elif a.what == "tune-budgets":
        tune_budgets(a.out, db)
    elif a.what == "mfma-ceiling":
        mfma_ceiling(a.out)
    elif a.what in ("collect-train", "collect-heldout"):
        done = collect(db, a.what.split("-")[1], a.budget)
        log("collect %s: %s" % (a.what, "complete" if done else "budget reached"))
    else:
        mlp(a.out, db)
    return 0


if __name__ == "__main__":
    sys.exit(main())
