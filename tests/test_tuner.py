"""Host-side checks of the autotuner (Sections 5 and 6): the Step-1 pruning
(Property 1, the convex hull, Heuristics 0-2), Step 2 with pruning as you go
(Property 3), the summaries of Table 2, and the interpolation of the
decision table (qr_tune, Section 6.1).

Pins: the Istanbul rows of Tables 2-6 (Appendix A and Section 6.4) as
printed, brute-force hulls on random point sets, and the interpolation
examples of Section 6.1.
"""
import itertools
import os

import numpy as np
import pytest

from paper_1102_5328_amd.tuner import heuristics as H
from paper_1102_5328_amd.tuner import step2 as S2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "istanbul_tables.txt")


def _golden():
    es, hrows, t2 = {}, [], {}
    with open(GOLDEN) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "ES":
                es[(int(w[1]), int(w[2]))] = float(w[3])
            elif w[0] in ("H0", "H1", "H2"):
                hrows.append((int(w[0][1]), int(w[1]), int(w[2]), float(w[4]), float(w[5]),
                              float(w[6]), float(w[7]), float(w[8])))
            elif w[0] == "T2":
                t2[int(w[1])] = tuple(float(x) for x in w[2:])
    return es, hrows, t2


# --------------------------------------------------------------- Table 2-6


def test_percentages_of_tables_4_to_6_from_printed_gflops():
    """PS/ES, PSPAYG/ES and PSPAYG/PS of every heuristic row from the
    printed GFLOP/s (the paper rounds after dividing unrounded rates, so the
    printed 2-decimal GFLOP/s reproduce the percentages to about 0.05)."""
    es, hrows, _ = _golden()
    assert len(hrows) == 48
    for h, n, c, ps, ps_es, pay, pay_es, pay_ps in hrows:
        ref = es[(n, c)]
        assert S2.percent(ps, ref) == pytest.approx(ps_es, abs=0.06), (h, n, c)
        assert S2.percent(pay, ref) == pytest.approx(pay_es, abs=0.06), (h, n, c)
        assert S2.percent(pay, ps) == pytest.approx(pay_ps, abs=0.06), (h, n, c)
        # An exhaustive search is never beaten; pruning never helps.
        assert ps <= ref + 1e-9 and pay <= ps + 1e-9


def test_table2_istanbul_summary():
    """Table 2 (Istanbul): average percentage and number of optima over the
    16 (N, ncores) points of Tables 4-6."""
    _, hrows, t2 = _golden()
    for h in (0, 1, 2):
        rows = [r for r in hrows if r[0] == h]
        assert len(rows) == 16
        exp = t2[h]
        for col, (avg_exp, opt_exp) in zip((4, 6, 7), ((exp[0], exp[1]), (exp[2], exp[3]),
                                                       (exp[4], exp[5]))):
            pct = [r[col] for r in rows]
            avg = round(sum(pct) / len(pct), 2)
            opt = sum(1 for p in pct if p >= 100.0)
            assert avg == pytest.approx(avg_exp, abs=0.011), (h, col)
            assert opt == opt_exp, (h, col)


def test_summary_function_matches_table2():
    """S2.summary on the printed GFLOP/s gives Table 2's optimum counts and
    averages within the rounding of the printed rates."""
    es, hrows, t2 = _golden()
    for h in (0, 1, 2):
        rows = [r for r in hrows if r[0] == h]
        got = [r[3] for r in rows]
        ref = [es[(r[1], r[2])] for r in rows]
        avg, opt, _ = S2.summary(got, ref)
        assert opt == int(t2[h][1])
        assert avg == pytest.approx(t2[h][0], abs=0.03)


# ------------------------------------------------------ Step 1 pruning


def _brute_upper_hull(pts):
    """Vertices of the upper hull by definition: a point is a vertex iff it
    lies strictly above every segment between two other points spanning its
    x (and is not dominated at its own x)."""
    out = []
    for p in pts:
        ok = True
        for a, b in itertools.combinations(pts, 2):
            if p in (a, b):
                continue
            lo, hi = (a, b) if a[0] <= b[0] else (b, a)
            if lo[0] <= p[0] <= hi[0]:
                if hi[0] == lo[0]:
                    if max(lo[1], hi[1]) >= p[1]:
                        ok = False
                    continue
                y = lo[1] + (hi[1] - lo[1]) * (p[0] - lo[0]) / (hi[0] - lo[0])
                if y >= p[1] - 1e-12:
                    ok = False
        if ok:
            out.append(p)
    return sorted(out)


@pytest.mark.parametrize("seed", range(6))
def test_upper_hull_brute_force(seed):
    rng = np.random.default_rng(seed)
    xs = sorted(rng.choice(np.arange(16, 520, 8), size=10, replace=False).tolist())
    pts = [(int(x), float(rng.uniform(10, 100))) for x in xs]
    hull = H.upper_hull(pts)
    top = max(pts, key=lambda p: (p[1], -p[0]))
    full = _brute_upper_hull(pts)
    assert hull == [p for p in full if p[0] <= top[0]]
    # Concave: slopes strictly decrease along the hull.
    sl = [(b[1] - a[1]) / (b[0] - a[0]) for a, b in zip(hull, hull[1:])]
    assert all(x > y for x, y in zip(sl, sl[1:]))


def test_property1_max_ib_envelope():
    step1 = {(64, 16): 10.0, (64, 32): 12.0, (64, 64): 11.0, (128, 16): 20.0, (128, 32): 20.0}
    env = H.max_ib_envelope(step1)
    assert env == {64: (32, 12.0), 128: (16, 20.0)}  # ties to the smaller IB


def _concave_step1(nbs, f):
    """Step-1 table whose Max-IB envelope is f(nb), with slower IBs around."""
    t = {}
    for nb in nbs:
        t[(nb, nb)] = f(nb) * 0.8
        t[(nb, max(16, nb // 4))] = f(nb)
        t[(nb, max(16, nb // 8))] = f(nb) * 0.9
    return t


def test_heuristics_on_a_concave_envelope():
    nbs = list(range(64, 513, 32))  # 15 tile orders
    step1 = _concave_step1(nbs, lambda nb: 300.0 * (1 - np.exp(-nb / 150.0)))
    hull = H.hull_points(step1)
    assert [p[0] for p in hull] == nbs  # strictly concave and increasing: all on the hull
    h0 = H.heuristic0(step1)
    assert h0 == [(nb, max(16, nb // 4)) for nb in nbs]
    # H1: on a concave hull the steepest segments come first -> first 8 by NB.
    assert H.heuristic1(step1) == h0[:8]
    # H2: 8 iso-segments of [64, 512] (width 56); each keeps its leftmost point.
    h2 = H.heuristic2(step1)
    edges = [64 + 56 * s for s in range(9)]
    exp = []
    for s in range(8):
        inseg = [nb for nb in nbs if edges[s] <= nb < edges[s + 1] or (s == 7 and nb == 512)]
        if inseg:
            exp.append(min(inseg))
    assert [p[0] for p in h2] == exp
    assert len(h2) <= 8 and len(H.heuristic1(step1)) <= 8


def test_hull_truncated_at_the_maximum():
    nbs = [64, 128, 192, 256, 320]
    vals = {64: 50.0, 128: 80.0, 192: 90.0, 256: 85.0, 320: 60.0}
    step1 = {(nb, 32): vals[nb] for nb in nbs}
    assert [p[0] for p in H.hull_points(step1)] == [64, 128, 192]


# ---------------------------------------------------------- Step 2 / PSPAYG


def _model_rate(M, N, nb, ib):
    """A synthetic performance landscape: small tiles win on small matrices,
    large tiles on large ones (the trade-off of Section 2.2)."""
    size = (M * N) ** 0.5
    par = 1.0 - np.exp(-size / (6.0 * nb))
    return 100.0 * (1.0 - 30.0 / nb) * par * (1.0 - 0.1 * ib / nb)


def test_pspayg_invariants():
    ps = [(64, 16), (96, 32), (128, 32), (192, 48), (256, 64), (384, 96), (512, 128)]
    shapes = [(n, n) for n in (512, 1024, 2048, 4096, 8192, 16384)]
    calls = []

    def meas(M, N, nb, ib):
        calls.append((M, N, nb, ib))
        return _model_rate(M, N, nb, ib), 1.0

    table_ps, t_ps = S2.step2(shapes, ps, meas, payg=False)
    n_ps = len(calls)
    calls.clear()
    table_pay, t_pay = S2.step2(shapes, ps, meas, payg=True)
    assert n_ps == len(ps) * len(shapes) and t_ps == n_ps
    assert len(calls) < n_ps and t_pay == len(calls)
    alive = list(ps)
    for shape in S2.order_sizes(shapes):
        res = table_pay[shape]
        assert sorted(res) == sorted(alive)
        # The best pair at each size survives the pruning of that size ...
        best = max(res, key=lambda p: res[p])
        after = S2.payg_prune(res, alive)
        assert best in after
        # ... and the survivors' rates do not increase with NB.
        rates = [res[p] for p in sorted(after)]
        assert all(a >= b for a, b in zip(rates, rates[1:]))
        alive = after
    # On this landscape (monotone in size) PSPAYG loses nothing.
    for shape in shapes:
        assert S2.decisions(table_pay)[shape] == S2.decisions(table_ps)[shape]


def test_payg_prune_strict():
    res = {(64, 16): 10.0, (128, 32): 10.0, (256, 64): 9.0}
    # Equal rates do not prune (strict >).
    assert S2.payg_prune(res, list(res)) == list(res)
    res[(128, 32)] = 10.5
    assert S2.payg_prune(res, list(res)) == [(128, 32), (256, 64)]


def test_aspect_classes_prune_separately():
    assert S2.aspect_class(65536, 256) == 8
    assert S2.aspect_class(4096, 4096) == 0
    assert S2.aspect_class(1024, 4096) == -2
    order = S2.order_sizes([(4096, 4096), (65536, 256), (1024, 1024), (16384, 64)])
    assert order == [(1024, 1024), (4096, 4096), (16384, 64), (65536, 256)]


def test_decision_table_roundtrip(tmp_path):
    dec = {(2000, 2000): (96, 32, 140.1), (4000, 4000): (168, 28, 250.0)}
    p = tmp_path / "t.txt"
    S2.write_table(str(p), dec, comment="two entries")
    lines = [l for l in p.read_text().splitlines() if not l.startswith("#")]
    assert lines == ["default 128 32", "entry 2000 2000 1 96 32 140.100",
                     "entry 4000 4000 1 168 28 250.000"]
