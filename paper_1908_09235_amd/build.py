"""Build the HIP library liblbm2p.so for gfx950 in the package directory."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# (source, extra flags): every kernel rounds every product and sum as
# written (no contraction into fused multiply-adds beyond the explicit
# ones), so that its results do not depend on where the compiler inlines
# the shared arithmetic.
UNITS = [("lbm2p.hip", ["-ffp-contract=off"]),
         ("batch.hip", ["-ffp-contract=off"]),
         ("noalloc.hip", ["-ffp-contract=off"]),
         ("launch_f64.hip", ["-ffp-contract=off"]),
         ("launch_f32.hip", ["-ffp-contract=off"])]
DEPS = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [
    os.path.join(ROOT, "include", "lbm2p.h")]
LIB = os.path.join(HERE, "liblbm2p.so")
ARCH = os.environ.get("LBM2P_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed-FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd))
    if verbose and r.stderr.strip():
        sys.stderr.write("\n".join(l for l in r.stderr.splitlines()
                                   if "packed-fp32-ops" not in l) + "\n")


def build(verbose: bool = False, extra=()) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src, flags in UNITS:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        _run(["hipcc", *FLAGS, *flags, *extra, "-c", "-o", obj,
              os.path.join(CSRC, src)], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(p) <= t for p in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
