"""Host-side pieces of the experiment flows: the MLP's features, the
training-set selection (held-out timings never train the model), the initial
weights, and the decision table written from a tuning run."""
import json
import math
import os

import numpy as np

from paper_1102_5328_amd import experiments as E
from paper_1102_5328_amd import inputs


def test_features_match_the_header_order():
    f = E.features(1024, 256, 128, 32, 2000)
    assert f == [math.log(1024), math.log(256), math.log(128), 0.25, math.log(2000)]


def test_training_rows_exclude_heldout():
    db = {
        "normal:100:100:64:16:1": {"gflops": 10.0, "M": 100, "N": 100, "nb": 64, "ib": 16,
                                   "batch": 1, "kind": "normal"},
        "heldout:300:300:64:16:1": {"gflops": 20.0, "M": 300, "N": 300, "nb": 64, "ib": 16,
                                    "batch": 1, "kind": "heldout"},
        "batched:128:64:128:16:2000": {"gflops": 30.0, "M": 85, "N": 47, "nb": 128, "ib": 16,
                                       "batch": 2000, "kind": "batched"},
        "illcond:4096:4096:64:16:1": {"gflops": 40.0, "M": 4096, "N": 4096, "nb": 64, "ib": 16,
                                      "batch": 1, "kind": "illcond"},
    }
    X, y = E._training_rows(db)
    assert X.shape == (2, 5)
    assert sorted(np.round(np.exp(y), 6).tolist()) == [10.0, 30.0]


def test_train_and_heldout_shapes_are_disjoint():
    train, test = E._shape_sets()
    assert len(test) == 200 and not set(train) & set(test)
    assert all(256 <= m <= 32768 and 256 <= n <= 32768 for m, n in test)
    assert test == inputs.log_uniform_shapes(200, seed=5)


def test_init_params_layout():
    p = E._init_params(0)
    assert p.shape == (8769,) and p.dtype == np.float32
    # Biases start at zero; weights within the He-uniform bound of their fan-in.
    for off, n in ((320, 64), (4480, 64), (8640, 64), (8768, 1)):
        assert np.all(p[off:off + n] == 0)
    assert np.max(np.abs(p[0:320])) <= math.sqrt(6 / 5)
    assert np.max(np.abs(p[384:4480])) <= math.sqrt(6 / 64)


def test_ship_table(tmp_path, monkeypatch):
    d = tmp_path / "run"
    d.mkdir()
    (d / "decision_table_h2r_pspayg.txt").write_text(
        "# x\ndefault 128 32\nentry 1024 1024 1 64 16 100.0\nentry 16384 16384 1 128 16 8000.0\n")
    (d / "batched_tune.json").write_text(json.dumps({"85x47": [128, 16, 58.7]}))
    out = tmp_path / "table.txt"
    entries = E.ship_table(str(d), str(out))
    assert len(entries) == 3
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert lines[0] == "default 128 16"  # the decision at the largest benchmarked size
    assert "entry 85 47 2000 128 16 58.700" in lines


def test_ship_table_carries_units(tmp_path):
    d = tmp_path / "run"
    d.mkdir()
    (d / "decision_table_h2r_units.txt").write_text(
        "default 128 16\nentry 4096 4096 1 64 16 2300.0 64\nentry 16384 16384 1 128 16 9200.0\n")
    out = tmp_path / "table.txt"
    E.ship_table(str(d), str(out), src_name="decision_table_h2r_units.txt")
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert "entry 4096 4096 1 64 16 2300.000 64" in lines
    assert "entry 16384 16384 1 128 16 9200.000" in lines
    assert lines[0] == "default 128 16"


def test_ship_table_domains_and_budgets(tmp_path):
    """Row-domain counts ride along as the eighth field; each tune-budgets
    output becomes a "budget C" section after the whole-device entries."""
    d = tmp_path / "run"
    d.mkdir()
    (d / "decision_table_h2r_pspayg.txt").write_text(
        "default 128 16\nentry 65536 256 1 128 16 1355.0 0 256\nentry 16384 16384 1 128 16 24000.0\n")
    (d / "decision_table_budget_64.txt").write_text("default 128 16\nentry 4096 4096 1 96 32 1500.0\n")
    (d / "decision_table_budget_128.txt").write_text("default 128 16\nentry 4096 4096 1 128 16 2500.0\n")
    out = tmp_path / "table.txt"
    E.ship_table(str(d), str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert "entry 65536 256 1 128 16 1355.000 0 256" in lines
    i64, i128 = lines.index("budget 64"), lines.index("budget 128")
    assert lines[i64 + 1] == "entry 4096 4096 1 96 32 1500.000"
    assert lines[i128 + 1] == "entry 4096 4096 1 128 16 2500.000"
    assert i64 < i128 and lines.index("entry 16384 16384 1 128 16 24000.000") < i64
