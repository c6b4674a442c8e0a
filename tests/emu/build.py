"""Builds the CPU emulation of the library's kernels (see hip/hip_runtime.h)
into a directory: `emu_qr` (tile QR, factor + apply, and batched) and
`emu_mlp` (the MLP kernels), both with AddressSanitizer, linked with the C
oracle for the comparisons. The device sources are compiled unchanged apart
from the few textual substitutions below (dynamic LDS and attributes the
host compiler does not take)."""
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1102_5328_amd", "csrc")
CLANG = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")
FLAGS = ["-std=c++20", "-g", "-O1", "-fsanitize=address", "-fno-omit-frame-pointer",
         "-Wno-unknown-attributes", "-I" + HERE, "-I" + os.path.join(ROOT, "include"),
         "-iquote", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:]))


def build(out_dir):
    os.makedirs(out_dir, exist_ok=True)
    s = open(os.path.join(CSRC, "tileqr_device.hip")).read()
    s = s.replace("extern __shared__ double lds_dyn[];", "double *lds_dyn = g_dyn_lds;")
    s = re.sub(r"__attribute__\(\(amdgpu_waves_per_eu\([^)]*\)\)\)", "", s)
    s = s.replace("typedef double d4 __attribute__((ext_vector_type(4)));", "typedef emu_d4 d4;")
    s = s.replace('asm volatile("" : "+v"(t));', "")
    dev = os.path.join(out_dir, "device_emu.cpp")
    open(dev, "w").write(s)
    m = open(os.path.join(CSRC, "tileqr_mlp.hip")).read()
    m = m.replace('#include "../../include/tileqr.h"', '#include "tileqr.h"')
    m = m.replace("extern __shared__ float smem[];", "float *smem = (float *)g_dyn_lds;")
    mlp = os.path.join(out_dir, "mlp_emu.cpp")
    open(mlp, "w").write(m)
    orc = os.path.join(out_dir, "oracle.o")
    _run(["gcc", "-O1", "-g", "-fsanitize=address", "-c", os.path.join(ROOT, "oracle", "oracle.c"),
          "-o", orc])
    glob = os.path.join(HERE, "globals.cpp")
    qr = os.path.join(out_dir, "emu_qr")
    _run([CLANG] + FLAGS + [dev, glob, os.path.join(HERE, "driver.cpp"),
                            os.path.join(CSRC, "plan.cpp"), orc, "-o", qr, "-lpthread"])
    ml = os.path.join(out_dir, "emu_mlp")
    _run([CLANG] + FLAGS + [mlp, glob, os.path.join(HERE, "mlp_driver.cpp"), orc, "-o", ml,
                            "-lpthread"])
    return qr, ml


if __name__ == "__main__":
    import sys
    print(build(sys.argv[1] if len(sys.argv) > 1 else "/tmp/tileqr_emu"))
