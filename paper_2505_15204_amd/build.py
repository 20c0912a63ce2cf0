"""Build libblink.so (the gfx950 HIP library behind include/blink.h) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libblink.so")
# (source, extra defines): split.hip is built once per split precision (1 = FP16, 2 = BF16),
# staged.hip once per precision form (0 = FP32).
UNITS = [("kernels.hip", []), ("persistent.hip", []), ("api.hip", []), ("correlate.hip", []),
         ("split.hip", ["-DBLINK_SPLIT_PREC=1"]), ("split.hip", ["-DBLINK_SPLIT_PREC=2"]),
         ("staged.hip", ["-DBLINK_STAGED_PREC=0"]), ("staged.hip", ["-DBLINK_STAGED_PREC=1"]),
         ("staged.hip", ["-DBLINK_STAGED_PREC=2"])]
SOURCES = sorted({os.path.join(CSRC, f) for f, _ in UNITS})

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # gfx950 only: no packed-FP32 instructions are generated
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln]
    return res.returncode, msgs


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every unit for gfx950 (in parallel) and link paper_2505_15204_amd/libblink.so."""
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="blink_build_") as tmpdir:
        objs, cmds = [], []
        for k, (src, defs) in enumerate(UNITS):
            obj = os.path.join(tmpdir, f"{k}_{os.path.splitext(src)[0]}.o")
            objs.append(obj)
            cmds.append([hipcc(), *HIPCC_FLAGS, *defs, "-I", INCLUDE, "-I", CSRC, "-c",
                         os.path.join(CSRC, src), "-o", obj])
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        all_msgs = []
        for (rc, msgs), cmd in zip(results, cmds):
            if rc != 0:
                raise RuntimeError(f"hipcc failed: {' '.join(cmd)}\n" + "\n".join(msgs))
            all_msgs += msgs
        tmp = LIB + ".tmp"
        rc, msgs = _run([hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp])
        if rc != 0:
            raise RuntimeError("link failed:\n" + "\n".join(msgs))
        all_msgs += msgs
    if verbose and all_msgs:
        print("\n".join(all_msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
