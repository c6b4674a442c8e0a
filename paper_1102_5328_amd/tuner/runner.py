"""GPU side of the tuner: measurements through the library, Step 1 on the
device, and the configuration-level flows (size sweep; pruned search vs
exhaustive search with reliability and tuning-time report).

Every factorization measured here is recorded (shape, NB, IB, batch,
GFLOP/s, seconds) in a JSON database; the searches read from it, so the
exhaustive search, the pruned searches and the learned cost model share one
set of runs. The tuning time of a method is the time of the runs it performs.
"""
import json
import os
import time

from .. import inputs
from . import heuristics as H
from . import step2 as S2

ENABLED_MAX_NB = 512  # largest tile order the library accepts


def config2_pairs(nbs=(64, 96, 128, 192, 256, 384, 512), ib_min=16, max_nb=ENABLED_MAX_NB):
    """The (NB, IB) grid of the square sweep: IB a divisor of NB, IB >= 16."""
    out = []
    for nb in nbs:
        if nb > max_nb:
            continue
        for ib in range(ib_min, nb + 1):
            if nb % ib == 0:
                out.append((nb, ib))
    return out


def domain_candidates(M, N, nb):
    """Row-domain counts p of the communication-avoiding tree tried for an
    M x N shape with tile order nb: the flat tree (p = 1) and, for tall
    shapes (M >= 16N, whose panels are long chains and whose steps are few),
    domains of 8, 4, 2 and 1 tile rows. (At M = 4N the merges' per-step
    synchronisation already costs more than the shorter chains save.)"""
    MT = -(-M // nb)
    out = [1]
    if M >= 16 * N:
        for h in (8, 4, 2, 1):
            p = -(-MT // h)
            if p > 1 and p not in out:
                out.append(p)
    return out


class Measurer:
    """Times tile QR factorizations on cuda:0 (median of `reps` runs after one
    warm-up, each on a fresh copy of the same seeded input), with a JSON
    cache keyed by (kind, M, N, NB, IB, batch)."""

    def __init__(self, db_path=None, reps=6, seed=0, verbose=True, offline=False):
        self.verbose = verbose
        self.offline = offline  # serve from the database only (no device)
        self.db_path = db_path
        self.reps = reps
        self.seed = seed
        self.db = {}
        if db_path and os.path.exists(db_path):
            with open(db_path) as f:
                self.db = json.load(f)
        self._shape = None
        self._A0 = None
        self._unsaved = 0  # new measurements since the last save
        # (units, torch stream): runs with that unit count go to a stream
        # restricted to those compute units (a caller's masked stream)
        self.masked = None

    def save(self):
        self._unsaved = 0
        if self.db_path:
            tmp = self.db_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.db, f)
            os.replace(tmp, self.db_path)

    @staticmethod
    def key(kind, M, N, nb, ib, batch=1, units=0, p=1):
        k = "%s:%d:%d:%d:%d:%d" % (kind, M, N, nb, ib, batch)
        return k + (":u%d" % units if units else "") + (":p%d" % p if p > 1 else "")

    def _input(self, kind, M, N):
        import torch
        if self._shape != (kind, M, N):
            self._A0 = None
            torch.cuda.empty_cache()
            if kind == "illcond":
                A = inputs.ill_conditioned(N, seed=self.seed)
                t = torch.empty((N, M), dtype=torch.float64, device="cuda").t()
                t.copy_(torch.from_numpy(A))
                self._A0 = t
            else:
                self._A0 = inputs.torch_normal(M, N, seed=self.seed)
            self._shape = (kind, M, N)
        return self._A0

    def measure_best_p(self, M, N, nb, ib, kind="normal", units=0):
        """The pair at its best row-domain count: (median GFLOP/s, seconds
        spent over every count tried, p)."""
        best, sec = None, 0.0
        for p in domain_candidates(M, N, nb):
            g, t = self.measure(M, N, nb, ib, kind=kind, units=units, p=p)
            sec += t
            if best is None or g > best[0]:
                best = (g, p)
        return best[0], sec, best[1]

    def measure(self, M, N, nb, ib, kind="normal", reps=None, units=0, p=1):
        """(median GFLOP/s, seconds spent) for one configuration; units > 0
        sizes the persistent grid for that many compute units, 0 for all; p
        row domains of the communication-avoiding tree (1: flat)."""
        k = self.key(kind, M, N, nb, ib, units=units, p=p)
        if k in self.db:
            r = self.db[k]
            return r["gflops"], r["seconds"]
        if self.offline:
            raise KeyError("not measured: " + k)
        import torch
        import paper_1102_5328_amd as tq
        reps = reps or self.reps
        A0 = self._input(kind, M, N)
        A = tq.colmajor(M, N)
        T = torch.empty(max(1, tq.T_size(M, N, nb, ib, p)), dtype=torch.float64, device="cuda")
        fl = tq.flops(M, N)
        tq.set_compute_units(units if units else torch.cuda.get_device_properties(0).multi_processor_count)
        st = self.masked[1] if (self.masked and units == self.masked[0]) else torch.cuda.current_stream()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        A.copy_(A0)
        torch.cuda.synchronize()
        tq.factor_ca(A, nb, ib, p, T, stream=st)
        tq.sync(st)
        g = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(reps):
            A.copy_(A0)
            torch.cuda.synchronize()
            e0.record(st)
            tq.factor_ca(A, nb, ib, p, T, stream=st)
            e1.record(st)
            tq.sync(st)
            g.append(fl / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        sec = time.perf_counter() - t_start
        tq.set_compute_units(0)
        med = S2.median(g)
        self.db[k] = {"gflops": med, "max": max(g), "runs": g, "seconds": sec, "M": M, "N": N,
                      "nb": nb, "ib": ib, "batch": 1, "kind": kind, "units": units, "p": p}
        if self.verbose:
            print("measured %s %dx%d nb=%d ib=%d units=%d p=%d: %.1f GFLOP/s (%.2f s)"
                  % (kind, M, N, nb, ib, units, p, med, sec), flush=True)
        del A, T
        self._unsaved += 1
        if self._unsaved >= 20:  # a run cut short keeps what it measured
            self.save()
        return med, sec


def step1_gpu(pairs, calls=50, flush_bytes=0):
    """Kernel benchmark of DSSRFB on every pair, one workgroup per CU. With
    flush_bytes = 0 the calls are timed together on warm tiles (No Flush);
    otherwise each call runs in its own launch after a write over
    flush_bytes of scratch memory that evicts the tiles (cold caches).
    Returns ({pair: gflops}, seconds)."""
    import paper_1102_5328_amd as tq
    import torch
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    t0 = time.perf_counter()
    for nb, ib in pairs:
        if flush_bytes > 0:
            sec = tq.ssrfb_bench_flush(nb, ib, calls, 0, flush_bytes)
        else:
            sec = tq.ssrfb_bench(nb, ib, calls, 0)
        out[(nb, ib)] = calls * ncu * 4.0 * nb ** 3 / sec / 1e9
    return out, time.perf_counter() - t0


# Step-2 size grid and test shapes of the tall/wide/square tuning run.
STEP2_GRID = [(1024, 1024), (2048, 2048), (4096, 4096), (8192, 8192), (16384, 16384),
              (16384, 256), (65536, 256), (16384, 1024), (65536, 1024),
              (8192, 2048), (16384, 4096), (4096, 1024),
              (1024, 4096), (4096, 16384)]
TEST_SHAPES = [("normal", 65536, 256), ("normal", 65536, 1024), ("normal", 16384, 4096),
               ("illcond", 4096, 4096),
               ("normal", 6000, 6000), ("normal", 12000, 12000), ("normal", 40000, 512),
               ("normal", 24000, 3000)]


def tune_search(measurer, out_dir, pairs=None, heuristics_=(0, 1, 2, "2r"), k=8, log=print,
                step1=None):
    """Pruned search (Step 1 -> heuristic -> Step 2 PS / PSPAYG) against the
    exhaustive search over the same candidates, on on-grid and off-grid test
    shapes; writes the decision tables and a JSON report. step1 = (rates,
    seconds) reuses a Step-1 table instead of running the kernel benchmark
    (with an offline measurer the whole analysis replays recorded runs)."""
    import paper_1102_5328_amd as tq
    pairs = pairs or config2_pairs()
    s1, t_step1 = step1 if step1 is not None else step1_gpu(pairs)
    log("step1 %.1f s: %s" % (t_step1, {"%dx%d" % p: round(v, 1) for p, v in s1.items()}))
    # each (NB, IB) is timed at its best row-domain count (the flat tree for
    # all but tall shapes); the tables record that count
    meas = lambda M, N, nb, ib: measurer.measure_best_p(M, N, nb, ib)[:2]
    best_p = lambda M, N, nb, ib, kind="normal": measurer.measure_best_p(M, N, nb, ib, kind=kind)[2]

    def with_p(dec):
        return {s: (d[0], d[1], d[2], 0, best_p(s[0], s[1], d[0], d[1])) for s, d in dec.items()}

    report = {"pairs": pairs, "step1_seconds": t_step1,
              "step1_gflops": {"%d,%d" % p: v for p, v in s1.items()}, "heuristics": {}}
    # Exhaustive search on the test shapes (the reference): every pair at
    # every row-domain count.
    es = {}
    for kind, M, N in TEST_SHAPES:
        res = {p: measurer.measure_best_p(M, N, p[0], p[1], kind=kind) for p in pairs}
        best = max(res, key=lambda p: res[p][0])
        es[(kind, M, N)] = (best, res[best][0], {p: v[0] for p, v in res.items()}, res[best][2])
        log("ES %s %dx%d: best %s p=%d %.1f GFLOP/s" % (kind, M, N, best, res[best][2], res[best][0]))
        measurer.save()
    # Exhaustive search over the size grid: its decisions and its tuning time
    # (the sum of the original runs' durations), the Table 1 analog.
    es_table, t_es = S2.step2(STEP2_GRID, pairs, meas, payg=False)
    measurer.save()
    S2.write_table(os.path.join(out_dir, "decision_table_es.txt"), with_p(S2.decisions(es_table)),
                   comment="exhaustive search")
    report["tuning_seconds"] = {"ES": t_es}
    for h in heuristics_:
        ps = H.preselect(s1, h, k)
        entry = {"preselected": ps}
        for payg in (False, True):
            table, t2 = S2.step2(STEP2_GRID, ps, meas, payg=payg)
            measurer.save()
            dec = with_p(S2.decisions(table))
            name = "PSPAYG" if payg else "PS"
            path = os.path.join(out_dir, "decision_table_h%s_%s.txt" % (h, name.lower()))
            S2.write_table(path, dec, comment="heuristic %s, %s" % (h, name))
            tq.tune_load(path)
            chosen, got, ref = [], [], []
            for kind, M, N in TEST_SHAPES:
                nb, ib, _ = tq.tune(M, N, 1)
                p = tq.tune_domains(M, N, 1)
                g = measurer.measure(M, N, nb, ib, kind=kind, p=p)[0]
                chosen.append([kind, M, N, nb, ib, g, p])
                got.append(g)
                ref.append(es[(kind, M, N)][1])
            avg, opt, pct = S2.summary(got, ref)
            report["tuning_seconds"]["H%s_%s" % (h, name)] = t_step1 + t2
            entry[name] = {"step2_seconds": t2, "avg_pct_of_ES": avg, "optimum": opt,
                           "n": len(got), "pct": pct, "chosen": chosen,
                           "table": {"%dx%d" % s: [d[0], d[1], d[2], d[4]] for s, d in dec.items()}}
            log("H%s %s: step2 %.1f s, avg %.2f%% of ES, optimum %d/%d" % (h, name, t2, avg, opt, len(got)))
        avg, opt, _ = S2.summary([c[5] for c in entry["PSPAYG"]["chosen"]],
                                 [c[5] for c in entry["PS"]["chosen"]])
        entry["PSPAYG_over_PS"] = {"avg": avg, "optimum": opt}
        report["heuristics"][str(h)] = entry
    report["ES"] = {"%s:%dx%d" % s: {"best": list(v[0]), "p": v[3], "gflops": v[1]}
                    for s, v in es.items()}
    with open(os.path.join(out_dir, "tuning_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    return report


def sweep_square(measurer, sizes=(2048, 4096, 8192, 16384), pairs=None, log=print):
    """GFLOP/s per (N, NB, IB) on square N(0,1) matrices."""
    pairs = pairs or config2_pairs()
    out = []
    for N in sizes:
        for nb, ib in pairs:
            g, sec = measurer.measure(N, N, nb, ib)
            out.append({"N": N, "nb": nb, "ib": ib, "gflops": g,
                        "max": measurer.db[measurer.key("normal", N, N, nb, ib)]["max"]})
            log("sweep N=%d nb=%d ib=%d %.1f GFLOP/s" % (N, nb, ib, g))
        measurer.save()
    return out
