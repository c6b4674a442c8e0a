"""Step-1 pruning of the (NB, IB) search space (Section 5 of the paper).

From the kernel benchmark of DSSRFB on every (NB, IB) pair:
  * Property 1 (orthogonal pruning): IB does not change the DAG's
    parallelism, so for each NB only the IB with the fastest kernel is kept
    (the "Max IB" envelope of Figure 5a).
  * Property 2 (convex hull): an optimal pair lies on the convex hull of
    that data set. Heuristic 0 keeps every hull point.
  * Heuristic 1 keeps the hull points that follow the steepest hull
    segments (at most 8); they cluster at small NB.
  * Heuristic 2 splits the NB axis into iso-segments and keeps the point
    after the steepest segment in each (at most 8 in total).

The paper's figure of the hull is missing from the text; readings used here
(also listed in the design notes):
  - the hull is the UPPER convex hull of the Max-IB points (x = NB, y = kernel
    GFLOP/s), truncated at the global maximum: larger tiles with no faster
    kernel only lose parallelism;
  - "steepness of a point" is the slope of the hull segment that ends at it;
    the leftmost hull point has no incoming segment and is always kept;
  - Heuristic 2 uses 8 segments of equal width over [NB_min, NB_max]; empty
    segments are skipped.
"""


def max_ib_envelope(step1):
    """Property 1. step1: {(nb, ib): gflops} -> {nb: (ib, gflops)}."""
    env = {}
    for (nb, ib), g in step1.items():
        if nb not in env or g > env[nb][1] or (g == env[nb][1] and ib < env[nb][0]):
            env[nb] = (ib, g)
    return env


def _cross(o, a, b):
    return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])


def upper_hull(points):
    """Upper convex hull of (x, y) points, left to right, truncated after the
    point of largest y (Andrew's monotone chain, upper part)."""
    pts = sorted(set(points))
    hull = []
    for p in pts:
        while len(hull) >= 2 and _cross(hull[-2], hull[-1], p) >= 0:
            hull.pop()
        hull.append(p)
    if not hull:
        return hull
    top = max(range(len(hull)), key=lambda i: (hull[i][1], -hull[i][0]))
    return hull[: top + 1]


def hull_points(step1):
    """Hull of the Max-IB envelope as [(nb, ib, gflops)], increasing nb."""
    env = max_ib_envelope(step1)
    h = upper_hull([(nb, g) for nb, (ib, g) in env.items()])
    return [(nb, env[nb][0], g) for nb, g in h]


def _incoming_slopes(hull):
    """Slope of the hull segment ending at each point (None for the first)."""
    out = [None]
    for a, b in zip(hull, hull[1:]):
        out.append((b[2] - a[2]) / float(b[0] - a[0]))
    return out


def heuristic0(step1):
    """Every point of the convex hull."""
    return [(nb, ib) for nb, ib, _ in hull_points(step1)]


def heuristic1(step1, k=8):
    """The leftmost hull point plus the points after the steepest segments."""
    hull = hull_points(step1)
    if not hull:
        return []
    slopes = _incoming_slopes(hull)
    rest = sorted(range(1, len(hull)), key=lambda i: (-slopes[i], hull[i][0]))
    keep = sorted([0] + rest[: max(0, k - 1)])
    return [(hull[i][0], hull[i][1]) for i in keep]


def heuristic2(step1, k=8):
    """Iso-segments of the NB axis; in each, the point after the steepest
    segment (the leftmost point of the first segment has none and is the
    segment's choice)."""
    hull = hull_points(step1)
    if not hull:
        return []
    env = max_ib_envelope(step1)
    lo, hi = min(env), max(env)
    slopes = _incoming_slopes(hull)
    width = (hi - lo) / float(k) if hi > lo else 1.0
    chosen = []
    for s in range(k):
        a, b = lo + s * width, lo + (s + 1) * width
        idx = [i for i, p in enumerate(hull) if (a <= p[0] < b) or (s == k - 1 and p[0] == hi)]
        if not idx:
            continue
        best = min(idx, key=lambda i: (0 if slopes[i] is None else 1,
                                       -(slopes[i] if slopes[i] is not None else 0.0), hull[i][0]))
        chosen.append(best)
    return [(hull[i][0], hull[i][1]) for i in sorted(set(chosen))]


def relaxed_property1(step1, nbs, tol=0.1, k=8):
    """For each tile order in `nbs`, every IB whose kernel rate is within
    `tol` of that order's best IB (Property 1 keeps only the best), at most
    k pairs in total, the fastest first within each order."""
    by_nb = {}
    for (nb, ib), g in step1.items():
        by_nb.setdefault(nb, []).append((g, ib))
    lists = []
    for nb in nbs:
        cand = sorted(by_nb.get(nb, []), key=lambda t: (-t[0], t[1]))
        if not cand:
            continue
        top = cand[0][0]
        lists.append([(nb, ib) for g, ib in cand if g >= (1.0 - tol) * top])
    out = []
    depth = 0
    while len(out) < k and any(depth < len(l) for l in lists):
        for l in lists:
            if depth < len(l) and len(out) < k:
                out.append(l[depth])
        depth += 1
    return sorted(out)


def heuristic2_relaxed(step1, k=8, tol=0.1):
    """GPU adaptation: the tile orders Heuristic 2 selects, each with every
    inner block whose DSSRFB rate is within `tol` of its best. On the GPU
    the inner block also sets the latency of the panel kernels on the
    critical path, which the DSSRFB benchmark does not see, so Property 1's
    single IB per NB is too strict there."""
    return relaxed_property1(step1, [nb for nb, _ in heuristic2(step1, k)], tol, k)


HEURISTICS = {0: heuristic0, 1: heuristic1, 2: heuristic2, "2r": heuristic2_relaxed}


def preselect(step1, heuristic=2, k=8):
    """Pre-selected set PS of (nb, ib) pairs."""
    if heuristic == 0:
        return heuristic0(step1)
    return HEURISTICS[heuristic](step1, k)
