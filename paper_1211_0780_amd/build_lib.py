"""Compile the gfx950 HIP library libxy.so in-tree (no JIT, no torch extension).

    python -m paper_1211_0780_amd.build_lib

Each source is compiled to an object with the common flags plus its own
(SOURCE_FLAGS), in parallel, and the objects are linked into the shared
library.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libxy.so")
SOURCES = ["xy_kernels.hip", "xy_or2.hip", "xy_capi.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions stay off: plain VALU float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]

# The plain fused over-relaxation substep (xy_or2.hip) takes the max-ILP
# instruction scheduler: 1.6 % less time per fused launch at L = 160 x 32 in
# an A/B run.  Built with it, other kernels need more registers and 11 of
# them (the measuring fused variants at 2, 4 and 5 columns per thread among
# them) lose occupancy, so they keep the default scheduler.
SOURCE_FLAGS = {
    "xy_or2.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags_signature():
    """The flags every source is compiled with, for hashing next to the sources."""
    return " ".join(HIPCC_FLAGS) + " | " + " ; ".join(
        f"{k}: {' '.join(v)}" for k, v in sorted(SOURCE_FLAGS.items()))


def build(verbose=False, extra=()):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    out_tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="xy_build_") as tmp:
        cmds = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmds.append([hipcc(), *HIPCC_FLAGS, *SOURCE_FLAGS.get(src, []), *extra, *inc, "-c",
                         os.path.join(CSRC, src), "-o", obj])
        if verbose:
            for cmd in cmds:
                print(" ".join(cmd), flush=True)
        with ThreadPoolExecutor(max_workers=len(cmds)) as pool:
            for f in [pool.submit(subprocess.check_call, c) for c in cmds]:
                f.result()
        link = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", out_tmp,
                *[c[c.index("-o") + 1] for c in cmds]]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
