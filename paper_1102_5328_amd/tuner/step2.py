"""Step 2 of the tuner (Section 6): benchmark the whole factorization on the
pre-selected pairs over a discretized size grid, with optional pruning as
you go (PSPAYG), and the summaries the paper reports.

* Discretization: sizes are benchmarked in increasing order; each run is
  repeated (6 times in the paper) and the median is the decision value
  (the paper does not say which statistic; the median is robust to a stray
  slow run).
* Property 3 (monotony) and PSPAYG: after all surviving pairs have been run
  at one size, a pair (NB2, IB2) is dropped for every larger size if some
  pair with NB1 > NB2 was strictly faster at that size.
* For non-square shapes the grid is ordered within each aspect class
  (M/N fixed) by size; pruning acts within a class.
* Interpolation (Section 6.1): a request is answered by the closest
  benchmarked configuration; that lookup is the library's qr_tune.
"""
import math
import statistics


def aspect_class(M, N):
    """Shapes of the same aspect ratio (rounded in log2) share a class."""
    return round(math.log2(M / float(N)))


def order_sizes(shapes):
    """Shapes grouped by aspect class, each class in increasing size."""
    return sorted(shapes, key=lambda s: (aspect_class(*s), s[0] * s[1]))


def payg_prune(results, alive):
    """Property 3: drop every pair beaten by a pair of larger NB.
    results: {pair: median gflops} at the current size."""
    keep = []
    for q in alive:
        beaten = any(p[0] > q[0] and results[p] > results[q] for p in alive if p in results)
        if not beaten:
            keep.append(q)
    return keep


def step2(shapes, ps, measure, payg=True):
    """Runs the pre-selected pairs over the shapes.

    measure(M, N, nb, ib) -> (median_gflops, seconds spent); it may serve
    from a cache of earlier measurements, the seconds are those of the
    original runs, so that the reported tuning time is what the method would
    have spent.
    Returns (table, seconds): table[(M, N)] = {pair: gflops} for the pairs
    run at that size.
    """
    table = {}
    seconds = 0.0
    alive_by_class = {}
    for shape in order_sizes(shapes):
        cls = aspect_class(*shape)
        alive = alive_by_class.setdefault(cls, list(ps))
        res = {}
        for pair in alive:
            g, t = measure(shape[0], shape[1], pair[0], pair[1])
            res[pair] = g
            seconds += t
        table[shape] = res
        if payg:
            alive_by_class[cls] = payg_prune(res, alive)
    return table, seconds


def decisions(table):
    """Best pair per benchmarked shape: {(M, N): (nb, ib, gflops)}."""
    out = {}
    for shape, res in table.items():
        pair = max(res, key=lambda p: (res[p], -p[0]))
        out[shape] = (pair[0], pair[1], res[pair])
    return out


def write_table(path, dec, batch=1, default=(128, 32), comment=None):
    """Decision table in the text format read by qr_tune_load."""
    with open(path, "w") as f:
        f.write("# tileqr decision table: entry M N batch NB IB gflops [units [p]]\n")
        if comment:
            for line in comment.splitlines():
                f.write("# %s\n" % line)
        f.write("default %d %d\n" % default)
        for (M, N), d in sorted(dec.items()):
            nb, ib, g = d[:3]
            units = d[3] if len(d) > 3 else 0
            p = d[4] if len(d) > 4 else 1
            if p > 1:
                f.write("entry %d %d %d %d %d %.3f %d %d\n" % (M, N, batch, nb, ib, g, units, p))
            elif units:
                f.write("entry %d %d %d %d %d %.3f %d\n" % (M, N, batch, nb, ib, g, units))
            else:
                f.write("entry %d %d %d %d %d %.3f\n" % (M, N, batch, nb, ib, g))


def median(xs):
    return statistics.median(xs)


def percent(a, b):
    """100 a / b rounded as the paper prints it (2 decimals)."""
    return round(100.0 * a / b, 2)


def summary(values, refs):
    """Average percentage and number of optima, as in Table 2: the mean of
    the per-test-point percentages 100 v/ref (each rounded to 2 decimals),
    and how many points reach 100 %."""
    pct = [percent(v, r) for v, r in zip(values, refs)]
    avg = round(sum(pct) / len(pct), 2) if pct else float("nan")
    opt = sum(1 for p in pct if p >= 100.0)
    return avg, opt, pct
