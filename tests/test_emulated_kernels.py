"""The library's HIP kernels compiled for the host and run under the CPU
emulation in tests/emu (every lane a host thread, LDS laid out as on the
device, MFMA with the measured gfx950 lane layout) with AddressSanitizer:
the index arithmetic of every task kind stays in bounds, and the results
match the oracle: R after sign normalisation, Q^T A = R, and Q (Q^T A) = A
(the reverse application). Covers every row-wave class (NB <= 128: one wave per
128-row slab of a column group; NB <= 256: two; NB <= 512: four), ragged
tiles, inner blocks that do not divide NB, the communication-avoiding tree, inner blocks wider than a
register panel (the T assembly across panels), the batched union DAG and
the MLP kernels. Runs on the CPU; slow (a few minutes in all)."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    import build as emu_build
    if not os.path.exists(emu_build.CLANG):
        pytest.skip("no host clang++ for the emulation")
    return emu_build.build(str(tmp_path_factory.mktemp("emu")))


def _run(args, timeout=600):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run(args, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, (args, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.parametrize("M,N,nb,ib", [
    (97, 130, 64, 12),     # wide, IB does not divide NB
    (200, 150, 128, 32),   # ragged both ways
    (110, 100, 96, 96),    # IB = NB wider than the 64-column register panel
    (260, 120, 128, 128),  # three tile rows, IB = NB = 128
    (150, 150, 136, 16),   # two row waves: LARFB/SSRFB with the register prefetch
    (280, 40, 256, 48),    # two row waves, T assembled over two register panels
    (520, 40, 512, 32),    # four row waves, T assembled over 16-column panels
    (384, 320, 128, 16),   # full 128-row tiles and 64-column strips: the straight-line update
    (384, 320, 128, 32),   # the same with two 16-column chunks per block
])
def test_tile_qr_emulated(emu, M, N, nb, ib):
    out = _run([emu[0], str(M), str(N), str(nb), str(ib)])
    assert "R_rel" in out


@pytest.mark.parametrize("M,N,nb,ib,p", [
    (300, 100, 64, 16, 2),   # two domains: chains, one merge per step
    (520, 200, 64, 16, 9),   # one tile row per domain, ragged: the tree alone
    (450, 130, 64, 12, 3),   # IB does not divide NB
    (330, 330, 64, 16, 2),   # square, trailing merges on every step
    (420, 100, 136, 16, 3),  # two row waves, ragged last domain head
])
def test_ca_tree_emulated(emu, M, N, nb, ib, p):
    # communication-avoiding variant: p row domains merged over a binary tree
    out = _run([emu[0], str(M), str(N), str(nb), str(ib), str(p)])
    assert "R_rel" in out


@pytest.mark.parametrize("M,N,nb,ib", [
    (200, 150, 64, 16),    # tall: the last steps have no LARFB (r > 0, c = 0)
    (150, 230, 64, 32),    # wide: the last step has no TSQRT (r = 0), ragged last strip
])
def test_program_order_decode_emulated(emu, M, N, nb, ib):
    # tasks decoded from the ticket in program order (no task list), as the
    # allocation-free entry point launches them
    out = _run([emu[0], "decode", str(M), str(N), str(nb), str(ib)])
    assert "R_rel" in out


def test_batched_emulated(emu):
    out = _run([emu[0], "batch", "3", "2"])
    assert "worst R_rel" in out


def test_mlp_emulated(emu):
    out = _run([emu[1], "100"])
    assert "grad rc=0" in out
