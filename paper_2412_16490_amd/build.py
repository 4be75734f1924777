"""Build the HIP library in-tree: paper_2412_16490_amd/libbodex_qp.so (gfx950).

Each kernel family is its own translation unit so the units compile in
parallel; the host part of the C ABI is one more unit.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
UNITS = ["bodex_qp.hip", "k_admm.hip", "k_finalize.hip", "k_finalize_sum.hip", "k_backward.hip",
         "k_backward_sum.hip", "k_detach.hip", "k_admm_cone.hip", "k_finalize_cone.hip",
         "k_backward_cone.hip", "k_hand.hip", "k_gpolish.hip", "k_finalize_chunk.hip"]
LIB = os.path.join(HERE, "libbodex_qp.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-pass-failed",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))] + [
        os.path.join(ROOT, "include", "bodex_qp.h")]


def _compile(unit, extra, verbose):
    obj = os.path.join(OBJDIR, unit.replace(".hip", ".o"))
    cmd = [HIPCC] + FLAGS + list(extra) + ["-c", os.path.join(CSRC, unit), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (unit, r.stderr[-6000:]))
    return obj, r.stderr


def build(verbose: bool = False, extra=()) -> str:
    """Compile every time it is called (the check that the code builds)."""
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        results = list(ex.map(lambda u: _compile(u, extra, verbose), UNITS))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _ in results] + ["-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
