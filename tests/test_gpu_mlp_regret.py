"""What the learned cost model gains over the method without it: an
ensemble trained on the GPU by the library's kernels on the recorded tuner
timings chooses (NB, IB) for the 200 held-out shapes (M, N log-uniform in
[256, 32768], seed 5); its regret against the exhaustive search (recorded
timings of every pair on every held-out shape) is compared with that of the
decision table alone. The candidates are the model's 14 pairs (tile orders
up to 256, IB of 16, 32 or 64), the exhaustive search is over them, and the
timings were taken with the shipped library on the whole device with the
flat tree; held-out shapes that the table answers with a tree are left out.
No factorization is timed here: the choices are scored with the recorded
exhaustive-search timings."""
import os

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DB = os.path.join(os.path.dirname(HERE), "paper_1102_5328_amd", "tuning", "mlp_timings.json")


def test_model_regret_against_exhaustive_search():
    import json
    from paper_1102_5328_amd import experiments as E
    with open(DB) as f:
        db = json.load(f)
    try:
        es = E.heldout_es(db)
    except KeyError:
        pytest.skip("held-out exhaustive-search timings are not all recorded")
    X, y = E._training_rows(db)
    params, fmean, fstd, ymean, ystd, losses, _ = E.train_ensemble(X, y)
    rep = E.evaluate(es, (params, fmean, fstd, ymean, ystd))
    print({k: v for k, v in rep.items() if k != "rows"})
    # every held-out shape but the tall ones the table answers with a tree
    assert rep["n_test"] + rep["n_tree_shapes_skipped"] == 200
    assert rep["n_test"] >= 150
    # The target: within 3 % of the exhaustive best on average, with the
    # pruned search as the fallback when the ensemble disagrees.
    assert rep["regret_mean"] <= 0.03
    # The gain: the model (with its fallback) does at least as well as the
    # decision table alone.
    assert rep["regret_mean"] <= rep["regret_table_only_mean"] + 1e-12
