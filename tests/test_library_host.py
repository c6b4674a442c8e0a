"""The C ABI on the host (no device needed): every entry point declared in
include/tileqr.h is exported by libtileqr.so; argument checking follows the
LAPACK info convention; the tile DAG (Section 2.1) has the task counts the
tiling fixes and its host-built order is a valid schedule; the flop model
shows the inner-blocking overhead of Section 2.2; qr_tune interpolates the
decision table as Section 6.1 describes.
"""
import ctypes
import os
import re

import pytest

import paper_1102_5328_amd as tq
from paper_1102_5328_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tileqr.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1102_5328_amd import build
        build.build()
    return _lib.lib()


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qr_[A-Za-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    raw = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing
    # ... and the binding describes each of them.
    assert sorted(_lib.SIGNATURES) == names


def test_version(lib):
    assert lib.qr_version().decode().startswith("tileqr")


# ------------------------------------------------------ argument checking


def test_factor_argument_errors(lib):
    f = lib.qr_factor
    p = ctypes.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert f(p, -1, 4, 4, 64, 16, p, None) == -2
    assert f(p, 4, -1, 4, 64, 16, p, None) == -3
    assert f(None, 4, 4, 4, 64, 16, p, None) == -1
    assert f(p, 8, 4, 7, 64, 16, p, None) == -4
    assert f(p, 8, 4, 8, 8, 4, p, None) == -5
    assert f(p, 8, 4, 8, 1024, 16, p, None) == -5
    assert f(p, 8, 4, 8, 64, 65, p, None) == -6
    assert f(p, 8, 4, 8, 64, -1, p, None) == -6
    assert f(p, 8, 4, 8, 64, 16, None, None) == -7


def test_factor_noalloc_argument_errors(lib):
    # the same checks as qr_factor, then the static scratch's size limit; all
    # of them return before any device call
    f = lib.qr_factor_noalloc
    p = ctypes.c_void_p(16)  # never dereferenced
    assert f(p, -1, 4, 4, 64, 16, p, None) == -2
    assert f(p, 4, -1, 4, 64, 16, p, None) == -3
    assert f(None, 4, 4, 4, 64, 16, p, None) == -1
    assert f(p, 8, 4, 7, 64, 16, p, None) == -4
    assert f(p, 8, 4, 8, 8, 4, p, None) == -5
    assert f(p, 8, 4, 8, 64, 65, p, None) == -6
    assert f(p, 8, 4, 8, 64, 16, None, None) == -7
    # 65536 x 16384 with NB = 16: 4096 x 1024 tiles, one strip each, plus
    # 1024 x 4096 panel counters: more than the 4 Mi ints of the scratch
    assert f(p, 65536, 16384, 65536, 16, 16, p, None) == 5  # TILEQR_ERR_TOO_LARGE
    assert f(p, 0, 16, 1, 64, 16, p, None) == 0  # empty: nothing to do


def test_ca_argument_errors(lib):
    # qr_factor_ca / qr_apply_Qt_ca: p in position 7; all checks return
    # before any device call
    f = lib.qr_factor_ca
    p = ctypes.c_void_p(16)
    assert f(p, -1, 4, 4, 64, 16, 2, p, None) == -2
    assert f(None, 4, 4, 4, 64, 16, 2, p, None) == -1
    assert f(p, 8, 4, 7, 64, 16, 2, p, None) == -4
    assert f(p, 8, 4, 8, 8, 4, 2, p, None) == -5
    assert f(p, 8, 4, 8, 64, 65, 2, p, None) == -6
    assert f(p, 8, 4, 8, 64, 16, -1, p, None) == -7
    assert f(p, 8, 4, 8, 64, 16, 2, None, None) == -8
    g = lib.qr_apply_Qt_ca
    assert g(p, 8, 4, 8, 64, 16, -3, p, p, 2, 8, None) == -7
    assert g(p, 8, 4, 8, 64, 16, 2, None, p, 2, 8, None) == -8
    assert g(p, 8, 4, 8, 64, 16, 2, p, None, 2, 8, None) == -9
    assert g(p, 8, 4, 8, 64, 16, 2, p, p, -2, 8, None) == -10
    assert g(p, 8, 4, 8, 64, 16, 2, p, p, 2, 4, None) == -11
    assert lib.qr_T_size_ca(8, 4, 64, 16, -1) == -5


def test_q_and_ls_argument_errors(lib):
    # qr_apply_Q(_ca), qr_form_Q_ca, qr_solve_ls_ca: every check before any
    # device call
    p = ctypes.c_void_p(16)
    f = lib.qr_apply_Q_ca
    assert f(None, 8, 4, 8, 64, 16, 1, p, p, 2, 8, None) == -1
    assert f(p, 8, 4, 8, 64, 16, -1, p, p, 2, 8, None) == -7
    assert f(p, 8, 4, 8, 64, 16, 1, None, p, 2, 8, None) == -8
    assert f(p, 8, 4, 8, 64, 16, 1, p, p, 2, 4, None) == -11
    g = lib.qr_apply_Q
    assert g(p, 8, 4, 8, 64, 16, None, p, 2, 8, None) == -7
    assert g(p, 8, 4, 8, 64, 16, p, p, -2, 8, None) == -9
    h = lib.qr_form_Q_ca
    assert h(p, 8, 4, 8, 64, 16, 1, p, p, 9, 8, None) == -10   # k > M
    assert h(p, 8, 4, 8, 64, 16, 1, p, None, 3, 8, None) == -9
    assert h(p, 8, 4, 8, 64, 16, 1, p, p, 3, 7, None) == -11
    assert h(p, 8, 4, 8, 64, 16, 1, None, p, 3, 8, None) == -8
    ls = lib.qr_solve_ls_ca
    assert ls(p, 4, 8, 4, 64, 16, 1, p, p, 2, 4, None) == -3    # N > M
    assert ls(p, 8, 4, 8, 64, 16, 1, p, None, 2, 8, None) == -9
    assert ls(p, 8, 4, 8, 64, 16, 1, p, p, 2, 3, None) == -11


def test_ca_T_size(lib):
    """The T buffer of p domains: the per-tile T factors, then one NB x NB
    reflector block and one IB x NB T factor per (step, domain)."""
    M, N, nb, ib = 1000, 300, 64, 16
    MT, NT = 16, 5
    KT = min(MT, NT)
    base = KT * MT * ib * nb
    assert tq.T_size(M, N, nb, ib) == base
    assert tq.T_size(M, N, nb, ib, 1) == base
    for p, D in ((2, 2), (5, 4), (16, 16), (100, 16)):  # h = ceil(MT/p), D = ceil(MT/h)
        assert tq.T_size(M, N, nb, ib, p) == base + KT * D * (nb * nb + ib * nb)


@pytest.mark.parametrize("M,N,nb,ib,p,workers,apply,nrhs", [
    (1000, 300, 64, 16, 3, 16, 2, 11),       # B <- Q B: the Q^T program reversed
    (700, 700, 64, 16, 1, 64, 2, 40),
    (1000, 200, 64, 16, 2, 64, False, 0),
    (1000, 200, 64, 16, 5, 7, False, 0),     # ragged last domain
    (1000, 200, 64, 16, 16, 256, False, 0),  # one row per domain
    (700, 150, 128, 32, 3, 32, True, 40),
    (600, 600, 64, 16, 4, 64, False, 0),
    (300, 700, 64, 32, 3, 16, True, 9),
    (4096, 128, 64, 16, 64, 16, False, 0),
])
def test_ca_plan_is_a_valid_schedule(lib, M, N, nb, ib, p, workers, apply, nrhs):
    """Tree DAGs: the ticket order replays with every wait satisfied, and the
    randomized parallel replay shows no hazard on tiles, the merges'
    reflector blocks or B."""
    for seed in (0, 1):
        nt, seq, stress = tq.plan_check(M, N, nb, ib, nrhs=nrhs, apply=apply, workers=workers,
                                        seed=seed, p=p)
        assert nt > 0 and seq == 0 and stress == 0


def test_ca_plan_task_multiset(lib):
    """Per step k of a 16 x 2 tile grid in domains of h = 4 rows: a GEQRT
    per domain head, a TSQRT per other row, and one merge per active domain
    but the first (the tree of E domains has E - 1 merges), each merge
    updating the trailing columns once."""
    tasks = tq.plan_tasks(1024, 128, 64, 16, p=4, workers=8)
    h, MT = 4, 16
    for k in range(2):
        rows = range(k, MT)
        heads = {i for i in rows if i == k or i % h == 0}
        ge = {int(t[1]) for t in tasks if t[0] == 0 and t[3] == k}
        ts = {int(t[1]) for t in tasks if t[0] == 1 and t[3] == k}
        tt = sorted(int(t[1]) for t in tasks if t[0] == 6 and t[3] == k)
        assert ge == heads
        assert ts == set(rows) - heads
        assert tt == sorted(i for i in heads if i != k)
        ttm = [(int(t[1]), int(t[2])) for t in tasks if t[0] == 7 and t[3] == k]
        assert sorted(i for i, j in ttm) == (tt if k == 0 else [])


def test_apply_argument_errors(lib):
    f = lib.qr_apply_Qt
    p = ctypes.c_void_p(16)
    assert f(None, 8, 4, 8, 64, 16, p, p, 2, 8, None) == -1
    assert f(p, -8, 4, 8, 64, 16, p, p, 2, 8, None) == -2
    assert f(p, 8, -4, 8, 64, 16, p, p, 2, 8, None) == -3
    assert f(p, 8, 4, 2, 64, 16, p, p, 2, 8, None) == -4
    assert f(p, 8, 4, 8, 8, 4, p, p, 2, 8, None) == -5
    assert f(p, 8, 4, 8, 64, 65, p, p, 2, 8, None) == -6
    assert f(p, 8, 4, 8, 64, 16, None, p, 2, 8, None) == -7
    assert f(p, 8, 4, 8, 64, 16, p, None, 2, 8, None) == -8
    assert f(p, 8, 4, 8, 64, 16, p, p, -2, 8, None) == -9
    assert f(p, 8, 4, 8, 64, 16, p, p, 2, 4, None) == -10


def test_other_argument_errors(lib):
    sec = ctypes.c_double()
    assert lib.qr_ssrfb_bench(8, 4, 1, 0, ctypes.byref(sec)) == -1
    assert lib.qr_ssrfb_bench(64, 65, 1, 0, ctypes.byref(sec)) == -2
    assert lib.qr_ssrfb_bench(64, 16, 0, 0, ctypes.byref(sec)) == -3
    assert lib.qr_ssrfb_bench(64, 16, 1, -1, ctypes.byref(sec)) == -4
    assert lib.qr_ssrfb_bench(64, 16, 1, 0, None) == -5
    f = lib.qr_ssrfb_bench_flush
    assert f(8, 4, 1, 0, 0, ctypes.byref(sec)) == -1
    assert f(64, 65, 1, 0, 0, ctypes.byref(sec)) == -2
    assert f(64, 16, 0, 0, 0, ctypes.byref(sec)) == -3
    assert f(64, 16, 1, -1, 0, ctypes.byref(sec)) == -4
    assert f(64, 16, 1, 0, -8, ctypes.byref(sec)) == -5
    assert f(64, 16, 1, 0, 0, None) == -6
    tf = ctypes.c_double()
    assert lib.qr_mfma_probe(0, 10, ctypes.byref(tf), None) == -1
    assert lib.qr_mfma_probe(9, 10, ctypes.byref(tf), None) == -1
    assert lib.qr_mfma_probe(2, 0, ctypes.byref(tf), None) == -2
    assert lib.qr_mfma_probe(2, 10, None, None) == -3
    assert lib.qr_T_size(-1, 4, 64, 16) == -1
    assert lib.qr_T_size(4, -1, 64, 16) == -2
    assert lib.qr_T_size(4, 4, 0, 16) == -3
    assert lib.qr_T_size(4, 4, 64, 0) == -4
    nb, ib, src = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert lib.qr_tune(-1, 4, 1, ctypes.byref(nb), ctypes.byref(ib), None) == -1
    assert lib.qr_tune(4, -1, 1, ctypes.byref(nb), ctypes.byref(ib), None) == -2
    assert lib.qr_tune(4, 4, 0, ctypes.byref(nb), ctypes.byref(ib), None) == -3
    assert lib.qr_tune(4, 4, 1, None, ctypes.byref(ib), None) == -4
    assert lib.qr_tune(4, 4, 1, ctypes.byref(nb), None, None) == -5
    assert lib.qr_tune_load(None) == -1
    assert lib.qr_tune_load(b"/nonexistent/table.txt") == 7


def test_T_size(lib):
    # KT * MT * IB * NB
    assert tq.T_size(512, 512, 128, 32) == 4 * 4 * 32 * 128
    assert tq.T_size(1000, 300, 96, 24) == 4 * 11 * 24 * 96
    assert tq.T_size(300, 1000, 96, 24) == 4 * 4 * 24 * 96
    assert tq.T_size(0, 10, 64, 16) == 0


# ---------------------------------------------------------------- tile DAG


@pytest.mark.parametrize("M,N,nb,counts", [
    (512, 512, 128, [4, 6, 6, 14]),
    (16384, 16384, 256, [64, 2016, 2016, 85344]),
    (16384, 16384, 64, [256, 32640, 32640, 5559680]),
    (65536, 256, 64, [4, 4086, 6, 6134]),
    (100, 300, 64, [2, 1, 7, 4]),
])
def test_dag_counts(lib, M, N, nb, counts):
    """GEQRT / TSQRT / LARFB / SSRFB counts: KT, sum_k (MT-k-1), sum_k (NT-k-1),
    sum_k (MT-k-1)(NT-k-1)."""
    assert tq.dag_counts(M, N, nb) == counts
    MT, NT = -(-M // nb), -(-N // nb)
    KT = min(MT, NT)
    assert counts == [KT, sum(MT - k - 1 for k in range(KT)), sum(NT - k - 1 for k in range(KT)),
                      sum((MT - k - 1) * (NT - k - 1) for k in range(KT))]


@pytest.mark.parametrize("M,N,nb,ib,workers,apply,nrhs", [
    (512, 512, 128, 32, 256, False, 0),
    (1000, 700, 96, 24, 64, False, 0),
    (700, 1000, 64, 16, 8, False, 0),
    (4096, 256, 64, 32, 256, False, 0),
    (777, 333, 64, 12, 32, True, 5),
])
def test_plan_is_a_valid_schedule(lib, M, N, nb, ib, workers, apply, nrhs):
    """The ticket order replays sequentially with every wait satisfied (seq =
    0 violations), and a randomized parallel replay with `workers` workers
    shows no read/write hazard on any tile (stress = 0)."""
    for seed in (0, 1):
        nt, seq, stress = tq.plan_check(M, N, nb, ib, nrhs=nrhs, apply=apply, workers=workers,
                                        seed=seed)
        assert nt > 0 and seq == 0 and stress == 0


def test_plan_task_multiset(lib):
    """Each tile task appears once per column strip; the order starts with
    GEQRT(0)."""
    tasks = tq.plan_tasks(512, 512, 128, 32)
    assert tuple(tasks[0][:4]) == (0, 0, 0, 0)
    types = sorted(set(int(t) for t in tasks[:, 0]))
    assert types == [0, 1, 2, 3]
    geqrt = {(int(t[1]), int(t[3])) for t in tasks if t[0] == 0}
    assert geqrt == {(k, k) for k in range(4)}
    ss = {(int(t[1]), int(t[2]), int(t[3])) for t in tasks if t[0] == 3}
    assert ss == {(i, j, k) for k in range(4) for i in range(k + 1, 4) for j in range(k + 1, 4)}


# ------------------------------------------------------------- flop model


def test_flops_formula(lib):
    assert tq.flops(1000, 1000) == pytest.approx(4.0 / 3.0 * 1e9)
    assert tq.flops(2000, 1000) == pytest.approx(2 * 2000 * 1e6 - 2e9 / 3)
    assert tq.flops(1000, 2000) == pytest.approx(2 * 2000 * 1e6 - 2e9 / 3)


def test_inner_blocking_overhead(lib):
    """Executed flops / algorithmic flops tends to 1 + IB/(4 NB) + 1/(2 NB)
    as the tile count grows: the T_s products add IB*NB^2 per DSSRFB on top
    of its 4 NB^3 (Section 2.2: IB = NB costs 25 % more), and the additions
    into the top tile 2 NB^2."""
    for nb, ib in ((128, 32), (64, 64), (128, 128)):
        lim = 1.0 + ib / (4.0 * nb) + 1.0 / (2.0 * nb)
        errs = [abs(tq.flops_executed(n, n, nb, ib) / tq.flops(n, n) - lim)
                for n in (4096, 16384, 65536)]
        assert errs[0] > errs[1] > errs[2]
        assert errs[2] < 5e-5


# ------------------------------------------------------------- qr_tune


def _table(tmp_path, entries, default=(128, 32)):
    p = tmp_path / "table.txt"
    with open(p, "w") as f:
        f.write("# test table\ndefault %d %d\n" % default)
        for e in entries:
            f.write("entry %d %d %d %d %d %.1f\n" % e)
    return str(p)


def test_tune_interpolation_examples(lib, tmp_path, monkeypatch):
    """Section 6.1: 2700 is answered by 2000 and 4200 by 4000 on a grid
    {1000, 2000, 4000, 6000}; a point between batch 4 and 8 (the paper's
    ncores axis) at 5 is answered by 4."""
    monkeypatch.delenv("TILEQR_NB", raising=False)
    monkeypatch.delenv("TILEQR_IB", raising=False)
    ents = [(1000, 1000, 1, 64, 16, 1), (2000, 2000, 1, 96, 32, 2), (4000, 4000, 1, 128, 32, 3),
            (6000, 6000, 1, 128, 64, 4), (2000, 2000, 4, 64, 32, 5), (2000, 2000, 8, 128, 16, 6)]
    tq.tune_load(_table(tmp_path, ents))
    try:
        assert tq.tune(2700, 2700, 1) == (96, 32, 1)
        assert tq.tune(4200, 4200, 1) == (128, 32, 1)
        assert tq.tune(1800, 1800, 5) == (64, 32, 1)
        assert tq.tune(10 ** 6, 10 ** 6, 1) == (128, 64, 1)
        # Equidistant in log space from 1000 and 4000: the larger wins.
        assert tq.tune(2000, 2000, 2)[:2] in ((96, 32), (64, 32))
        ents2 = [(1000, 1000, 1, 64, 16, 1), (4000, 4000, 1, 128, 32, 3)]
        tq.tune_load(_table(tmp_path, ents2))
        assert tq.tune(2000, 2000, 1) == (128, 32, 1)
        # Environment override.
        monkeypatch.setenv("TILEQR_NB", "96")
        monkeypatch.setenv("TILEQR_IB", "48")
        assert tq.tune(2000, 2000, 1) == (96, 48, 3)
    finally:
        monkeypatch.delenv("TILEQR_NB", raising=False)
        monkeypatch.delenv("TILEQR_IB", raising=False)
        tq.tune_load(_table(tmp_path, []))
    # An empty table: the default, source 0.
    assert tq.tune(5000, 5000, 1) == (128, 32, 0)


def test_tune_budget_sections_and_domains(lib, tmp_path, monkeypatch):
    """Entries under "budget C" serve callers limited to C compute units; a
    caller without a setting (the whole device) takes the "all" section when
    there is one, else the nearest budget. The optional eighth field of an
    entry is the tree's domain count, which p = 0 resolves to."""
    monkeypatch.delenv("TILEQR_NB", raising=False)
    monkeypatch.delenv("TILEQR_IB", raising=False)
    p = tmp_path / "budget.txt"
    p.write_text("default 128 32\n"
                 "entry 4000 4000 1 128 16 9.0 192\n"
                 "entry 65536 256 1 64 16 1.0 0 128\n"
                 "budget 64\n"
                 "entry 4000 4000 1 96 32 5.0\n")
    tq.tune_load(str(p))
    try:
        assert tq.tune(4000, 4000, 1) == (128, 16, 1)
        assert tq.tune_units(4000, 4000, 1) == 192
        MT, KT, D = 1024, 4, 128
        assert tq.T_size(65536, 256, 64, 16, 0) == KT * MT * 16 * 64 + KT * D * (64 * 64 + 16 * 64)
        p.write_text("budget 64\nentry 4000 4000 1 96 32 5.0\n")
        tq.tune_load(str(p))
        assert tq.tune(4000, 4000, 1) == (96, 32, 1)
        p.write_text("budget -3\nentry 4000 4000 1 96 32 5.0\n")
        assert lib.qr_tune_load(str(p).encode()) == 7
        p.write_text("entry 4000 4000 1 96 32 5.0 0 0\n")  # p < 1
        assert lib.qr_tune_load(str(p).encode()) == 7
    finally:
        tq.tune_load(_table(tmp_path, []))


def test_tune_load_rejects_malformed(lib, tmp_path):
    p = tmp_path / "bad.txt"
    p.write_text("entry 100 100 1 8 4 1.0\n")  # NB below 16
    assert lib.qr_tune_load(str(p).encode()) == 7
    p.write_text("garbage\n")
    assert lib.qr_tune_load(str(p).encode()) == 7


def test_shipped_decision_table(lib):
    """The table the benchmark loads parses, and qr_tune answers from it:
    the measured best at 16384^2, and a batch-class entry for a matrix of
    the 2000-matrix batch."""
    path = os.path.join(ROOT, "paper_1102_5328_amd", "tuning", "decision_table.txt")
    tq.tune_load(path)
    try:
        entries = {}
        for line in open(path):
            w = line.split()
            if w and w[0] == "entry":
                entries[(int(w[1]), int(w[2]), int(w[3]))] = (int(w[4]), int(w[5]))
        assert tq.tune(16384, 16384, 1)[:2] == entries[(16384, 16384, 1)]
        assert tq.tune(16384, 16384, 1)[2] == 1
        batch = [k for k in entries if k[2] > 1]
        assert batch
        m, n, b = batch[0]
        assert tq.tune(m, n, b)[:2] == entries[(m, n, b)]
    finally:
        tq.tune_load(os.devnull)


def test_tune_set_model_argument_errors(lib):
    import numpy as np
    F = ctypes.POINTER(ctypes.c_float)
    I = ctypes.POINTER(ctypes.c_int)
    p = np.zeros(8769, np.float32)
    fm = np.zeros(5, np.float32)
    fs = np.ones(5, np.float32)
    good = np.array([64, 16, 128, 32], np.int32)
    bad = np.array([64, 16, 128, 200], np.int32)
    f = lib.qr_tune_set_model
    P = lambda a: a.ctypes.data_as(F)
    assert f(P(p), 65, P(fm), P(fs), 0.0, 1.0, good.ctypes.data_as(I), 2) == -1
    assert f(None, 1, P(fm), P(fs), 0.0, 1.0, good.ctypes.data_as(I), 2) == -2
    assert f(P(p), 1, None, P(fs), 0.0, 1.0, good.ctypes.data_as(I), 2) == -3
    fz = fs.copy()
    fz[3] = 0.0
    assert f(P(p), 1, P(fm), P(fz), 0.0, 1.0, good.ctypes.data_as(I), 2) == -4
    assert f(P(p), 1, P(fm), P(fs), 0.0, 1.0, bad.ctypes.data_as(I), 2) == -7
    assert f(P(p), 1, P(fm), P(fs), 0.0, 1.0, None, 2) == -7
    assert f(None, 0, None, None, 0.0, 1.0, None, 0) == 0


def test_tune_units_from_table(lib, tmp_path, monkeypatch):
    """The optional units column: the nearest entry's unit count sizes the
    grid (0 or absent: all units); qr_set_compute_units is not needed."""
    p = tmp_path / "units.txt"
    p.write_text("default 128 16\nentry 4096 4096 1 64 16 2300.0 64\n"
                 "entry 16384 16384 1 128 16 9200.0 0\nentry 2048 2048 1 64 16 450.0\n")
    tq.tune_load(str(p))
    try:
        assert tq.tune_units(4000, 4200, 1) == 64
        assert tq.tune_units(16000, 16000, 1) == 0
        assert tq.tune_units(2000, 2000, 1) == 0
        assert tq.tune(4000, 4200, 1) == (64, 16, 1)
        assert lib.qr_tune_units(-1, 4, 1, ctypes.byref(ctypes.c_int())) == -1
        assert lib.qr_tune_units(4, 4, 1, None) == -4
        p.write_text("entry 4096 4096 1 64 16 2300.0 -3\n")
        assert lib.qr_tune_load(str(p).encode()) == 7
    finally:
        tq.tune_load(os.devnull)
