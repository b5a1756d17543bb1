"""Build libstamp.so (gfx950) in-tree with hipcc.

Run as ``python paper_2310_01775_amd/build.py`` (a plain script: it must not
import the package, whose __init__ loads the library being built); always
recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libstamp.so")
SOURCES = ["stamp_api.hip", "rollout.hip", "svgd.hip", "median.hip", "phi16.hip", "mlp.hip", "structured.hip", "phi32.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 VALU ops stay off: scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit mul+add fusion: the same source must round the same way in
    # every kernel it is inlined into (checkpoint replay repeats the forward
    # bit for bit); fusion is written out with fmaf where wanted
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


# per-source additions: the BF16 contraction turns its Gram products into
# kernel values with VALU code, which then reads them from VGPRs directly
EXTRA = {"phi16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link."""
    with tempfile.TemporaryDirectory(prefix="stamp_build_") as tmpdir:
        objs, procs = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, s.replace(".hip", ".o"))
            cmd = [HIPCC, *FLAGS, *EXTRA.get(s, []), "-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = False
        for s, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                sys.stderr.write(out)
                failed = True
            elif verbose and out.strip():
                sys.stderr.write(out)
        if failed:
            raise RuntimeError("hipcc failed building libstamp.so")
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libstamp.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
