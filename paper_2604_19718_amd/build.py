"""Build libcdz.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["cdz_host.hip", "cdz_fwd.hip", "cdz_out.hip", "cdz_sample.hip", "cdz_batch.hip", "cdz_freq.hip", "cdz_mfe.hip",
           "cdz_tensor.hip"]
OUT = os.path.join(HERE, "libcdz.so")


def hipcc_cmd(out: str = OUT):
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES
            if os.path.exists(os.path.join(HERE, "csrc", s))]
    return (["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
             # packed FP32 VALU forms are kept out of every kernel
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
             "-o", out] + srcs)


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    r = subprocess.run(hipcc_cmd(tmp), capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libcdz.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
