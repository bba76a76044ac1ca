#!/usr/bin/env python3
"""Wall time of the FP64 CPU oracle on the seeded workloads (test
infrastructure: the CPU baseline the GPU path is reported beside).

For workloads 1-3 it times, with steady wall clock, the forward pass (log Z),
the forward + outside pass with all marginals, and the exact sampler, and
prints one JSON line per workload with the thread count and the CPU model.

Usage: OMP_NUM_THREADS=<t> python oracle/time_oracle.py [--workloads 1,2,3]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2604_19718_amd import inputs as I  # noqa: E402

SAMPLES = {1: 100, 2: 1000, 3: 1000}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="1,2,3")
    a = ap.parse_args()
    oracle.build(force=False)
    for k in (int(x) for x in a.workloads.split(",")):
        prob, en = I.workload(k)
        n = prob.n
        t0 = time.perf_counter()
        lz = oracle.logz(prob, en)
        t1 = time.perf_counter()
        oracle.marginals(prob, en)
        t2 = time.perf_counter()
        oracle.sample(prob, en, I.sampler_seed(k), SAMPLES[k])
        t3 = time.perf_counter()
        cells = n * (n + 1) / 2
        print(json.dumps({
            "workload": k, "n_nt": n, "threads": oracle.num_threads(), "cpu": cpu_model(),
            "logical_cpus": os.cpu_count(), "logz": lz,
            "s_forward": t1 - t0, "s_forward_outside_marginals": t2 - t1,
            "s_samples": t3 - t2, "samples": SAMPLES[k],
            "cells_per_s_forward_outside": cells / (t2 - t1),
        }), flush=True)


if __name__ == "__main__":
    main()
