"""Empirical (NB, IB) tuner of the tile QR: the two-step pruned search of
the paper (Step 1 kernel benchmark + convex-hull heuristics, Step 2 whole-QR
benchmark with prune-as-you-go) and the decision table read by qr_tune.

Modules: heuristics (Step 1 pruning), step2 (Step 2 and the summaries),
runner (measurements on the device and the end-to-end flows)."""
