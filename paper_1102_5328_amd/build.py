"""Builds libtileqr.so (HIP kernels + host runtime + C ABI) in-tree for gfx950.

    python -m paper_1102_5328_amd.build
"""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtileqr.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["tileqr_device.hip", "tileqr_mlp.hip", "tileqr_probe.hip", "tileqr_api.cpp", "plan.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-Wno-unused-value"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Register budget of every kernel: 256 VGPRs (two waves per SIMD), no
# accumulation registers and no scratch (private memory for spills).
MAX_VGPRS = 256


def kernel_resources(remarks):
    """Parses -Rpass-analysis=kernel-resource-usage remarks into
    {kernel: {"VGPRs": n, "AGPRs": n, "ScratchSize": n}}."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and cur is not None:
            cur[m.group(1).split()[0]] = int(m.group(2))
    return out


def check_resources(res, src):
    bad = []
    for k, r in res.items():
        if r.get("VGPRs", 0) > MAX_VGPRS or r.get("AGPRs", 0) > 0 or r.get("ScratchSize", 0) > 0:
            bad.append("%s: %s" % (k, r))
    if bad:
        raise RuntimeError("kernel register budget exceeded in %s:\n  %s" % (src, "\n  ".join(bad)))


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + DEVICE
    if src.endswith(".hip"):
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    if src.endswith(".hip"):
        res = kernel_resources(r.stderr)
        if not res:
            raise RuntimeError("no kernel resource report for %s" % src)
        check_resources(res, src)
        with open(os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".resources.txt"), "w") as f:
            for k in sorted(res):
                f.write("%s %s\n" % (k, res[k]))
    return obj


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
