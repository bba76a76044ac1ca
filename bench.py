#!/usr/bin/env python3
"""Benchmark of the codon-constrained McCaskill hot path on one MI355X.

A step is one pass of the whole path over one protein of 300 residues
(900 nt, codon and codon-pair weights): FP32-scaled forward (log Z), outside
pass with pair/base/codon/codon-pair marginals, and 1000 exact joint samples.
Inputs are seeded and synthetic (see paper_2604_19718_amd/inputs.py).

Prints ONE JSON line.  `value` is DP cells per second of forward + outside,
n(n+1)/2 / (t_forward + t_outside), from HIP events on the library's stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N_SAMPLES = 1000
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_fwd(d: np.ndarray, w: int) -> float:
    """Bytes the forward diagonal kernel must move, summed over all launches:
    for every cell (i, j) the O(n) split reads the d_i rows of Qm and the d_j
    rows of Qm1L over K = sum_{u=i+5}^{j-4} d_{u-1} states, and writes the five
    d_i x d_j blocks Qb, Qm1, Qm1p, QmX, Qm.  Padding never counts."""
    n = len(d)
    P = np.concatenate([[0], np.cumsum(d)])
    tot = 0.0
    for dl in range(4, n):
        i = np.arange(0, n - dl)
        j = i + dl
        K = np.where(dl >= 9, P[np.minimum(j - 4, n)] - P[np.minimum(i + 4, n)], 0)
        tot += float(np.sum((d[i] + d[j]) * K) + 5 * np.sum(d[i] * d[j]))
    return tot * w


def algorithmic_bytes_out(d: np.ndarray, w: int) -> float:
    """Bytes the outside diagonal kernel must move, summed over all launches:
    for every cell (i, j) with j - i >= 4 the two split pulls (the d_i rows of
    QmX' and the d_j rows of Qm1L over the states of positions j+5..n-1; the
    d_{i-1} rows of Qm and the d_j rows of QmX' over the states of positions
    0..i-5) and the adjoint blocks it writes: seven at (i, j) (Qb', Qm1',
    Qm1p', QmX' and its transpose, Qm', U'), Qm1L' at (i-1, j), DI' at
    (i-1, j+1), G' and F' at (i+1, j-1).  Cells with j - i < 4 write their six
    zero blocks and U'.  Padding never counts."""
    n = len(d)
    P = np.concatenate([[0], np.cumsum(d)])
    dz = np.concatenate([d, [0]])  # d of position n (absent) reads as 0
    tot = 0.0
    for dl in range(0, n):
        i = np.arange(0, n - dl)
        j = i + dl
        own = d[i] * d[j]
        if dl < 4:
            tot += float(7 * np.sum(own))
            continue
        KR = np.where(j + 5 <= n - 1, P[n] - P[np.minimum(j + 5, n)], 0)
        KL = np.where(i >= 5, P[np.maximum(i - 4, 0)], 0)
        dim1 = np.where(i >= 1, d[np.maximum(i - 1, 0)], 0)
        djp1 = dz[np.minimum(j + 1, n)]
        tot += float(np.sum((d[i] + d[j]) * KR) + np.sum((dim1 + d[j]) * KL))
        tot += float(np.sum(7 * own + dim1 * d[j] + dim1 * djp1 + 2 * d[i + 1] * d[j - 1]))
    return tot * w


FP64_ALU_PEAK_TOPS = 78.6 / 2  # FP64 vector adds or minima per second (TOP/s): half the FMA flop rate


def algorithmic_ops_mfe(d: np.ndarray) -> float:
    """(min, +) operations of the MFE diagonal kernel, summed over all cells
    (each add and each minimum counted once): for every cell (i, j) with
    j - i >= 4, each bulge window (run, edge, inner pair: two adds and a
    minimum per inner slot pair, one add for the loop energy) and interior
    window (per slot c of l+1: an add and a minimum per slot of k-1, then an
    add and a minimum; one add for the energy) at every outer slot pair
    (a, dd), and the split (two adds and a minimum per (s, s2, t, t2) over
    u = i+5..j-4).  The O(1) terms of the pair and branch blocks are left out."""
    n = len(d)
    dz = np.concatenate([d, [0]])
    # per u: d_{u-1} d_u, prefix-summed
    du = np.concatenate([[0], d[:-1] * d[1:]])  # du[u] = d[u-1] d[u] for u >= 1
    Pu = np.concatenate([[0], np.cumsum(du)])   # Pu[x] = sum_{u < x} du[u]
    tot = 0.0
    for dl in range(4, n):
        i = np.arange(0, n - dl)
        j = i + dl
        outer = d[i + 1] * d[j - 1]
        for l1 in range(0, 31):
            for l2 in range(0, 31 - l1):
                if (l1 == 0 and l2 == 0) or l1 + l2 > dl - 6:
                    continue
                k, l = i + 1 + l1, j - 1 - l2
                if l2 == 0:
                    per = dz[k - 1] * dz[k] * 3 + 1
                elif l1 == 0:
                    per = dz[l] * dz[l + 1] * 3 + 1
                else:
                    per = dz[l + 1] * (dz[k - 1] * 2 + 2) + 1
                tot += float(np.sum(outer * per))
        if dl >= 9:
            K = Pu[j - 3] - Pu[i + 5]  # u = i+5..j-4
            tot += float(np.sum(d[i] * d[j] * K * 3))
    return tot


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "cdz_out_diag_float_900nt_traffic.md")


# the sources each diagonal kernel is compiled from
KERNEL_SOURCES = {
    "out": ["paper_2604_19718_amd/csrc/cdz_out.hip", "paper_2604_19718_amd/csrc/cdz_internal.h",
            "paper_2604_19718_amd/csrc/cdz_dev.h", "include/cdz.h"],
    "fwd": ["paper_2604_19718_amd/csrc/cdz_fwd.hip", "paper_2604_19718_amd/csrc/cdz_dev.h"],
    "tensor": ["paper_2604_19718_amd/csrc/cdz_tensor.hip"],
}
TENSOR_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "tz_prop_float_900nt_traffic.md")


def source_sha256(kernel: str = "out") -> str:
    """Hash of the sources a diagonal kernel is compiled from (the key under which
    its traffic counters were taken)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        h.update(os.path.basename(rel).encode())
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str = "out", path: str = TRAFFIC_PROFILE):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs (scaled by a copy kernel of known size), or None when those counters
    were taken on other kernel sources."""
    try:
        with open(path) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines() if ": " in line and not line.startswith(("|", "`", "#")))
        if kv.get("source_sha256", "").strip() != source_sha256(kernel):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def run_step(B, h, prob, seed):
    B.cdz_reset(h)
    out = B.cdz_marginals(h, prob)
    if hasattr(B.lib(), "cdz_sample"):
        B.cdz_sample(h, prob, seed, N_SAMPLES)
    return out


def cpu_baseline(prob, en):
    """The FP64 oracle (forward + reverse-mode marginals) on a bounded sample:
    the first 150 residues (450 nt) of the same protein."""
    import oracle
    from paper_2604_19718_amd import inputs as I
    m = 150
    sub = I.Problem(prob.prot[:m], prob.theta1[:m], None if prob.theta2 is None else prob.theta2[:m])
    n = 3 * m
    t0 = time.perf_counter()
    oracle.marginals(sub, en)
    dt = time.perf_counter() - t0
    return {"value": n * (n + 1) / 2 / dt, "unit": "DP cells/s (forward+outside)",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"forward + outside marginals of the first {m} residues ({n} nt) of the "
                      f"900-nt protein, {dt:.1f} s"}


def tensor_cpu_baseline():
    """The tensor-model oracle (FP64, 8 threads) on the 100-residue (300-nt)
    protein of workload 2: the 900-nt pass takes about 45 s on 8 cores."""
    import oracle
    from paper_2604_19718_amd import inputs as I
    prob, model = I.tensor_workload(2)
    t0 = time.perf_counter()
    oracle.tensor_logz(prob, model)
    dt = time.perf_counter() - t0
    return {"value": 1e3 * dt, "unit": "ms per pass", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one FP64 pass over the {prob.n}-nt protein of workload 2, {dt:.2f} s"}


MFMA_FP32_PEAK_TFS = 157.3
MFMA_FP64_PEAK_TFS = 78.6


def tensor_prop_algorithmic(sig: np.ndarray, g: int, elt: int):
    """Algorithmic bytes and useful flops of every propagation launch j of the
    tensor-model pass, summed over j = 1..n.  Launch j reads, for each row of
    position blocks p < j, the row from its own block's start to off[j] (the
    triangle of Q, identity diagonal blocks included), reads the fold row
    block j (gamma Sigma_j rows of off[j]) and writes gamma Sigma_j columns of
    off[j] rows; flops = 2 * (triangle entries) * gamma Sigma_j."""
    n = len(sig) - 1
    h = g * sig.astype(np.int64)
    off = np.concatenate([[0], np.cumsum(h)])
    tot_b = tot_f = 0.0
    for j in range(1, n + 1):
        R = off[j]
        tri = float(np.sum(h[:j] * (R - off[:j])))
        w = float(h[j])
        tot_b += (tri + 2.0 * w * R) * elt
        tot_f += 2.0 * tri * w
    return tot_b, tot_f


def tensor_leg(B, I, h32, h64, steps):
    """The tensor-based model's free energy (Sections 3b-3c) of the 900-nt
    protein with synthetic (gamma 9, xi 1) parameters: FP32 (the paper's
    precision) and FP64 passes, and the propagation kernel against its
    roofline from per-launch HIP events."""
    prob, model = I.tensor_workload(3)
    sig = B.cdz_tensor_dims(prob)
    out = {"workload": "tensor-model free energy, 300 residues (900 nt), single-codon train with codon "
                       "bonuses, synthetic V/B/S of gamma 9, xi 1",
           "sum_sigma": int(sig.sum()), "q_rows": int(9 * sig.sum())}
    for name, hh in (("fp32", h32), ("fp64", h64)):
        B.cdz_tensor_logz(hh, model, prob)  # warm-up
        ts = []
        for _ in range(steps):
            lz, _ = B.cdz_tensor_logz(hh, model, prob)
            ts.append(B.cdz_last_timings(hh)[0])
        out[f"ms_{name}"] = float(np.median(ts))
        out[f"logz_{name}"] = lz
        print(f"# tensor {name} {out[f'ms_{name}']:.2f} ms logz {lz:.6f}", file=sys.stderr, flush=True)
    B.cdz_set_profiling(h32, True)
    B.cdz_tensor_logz(h32, model, prob)
    tm = B.cdz_last_timings(h32)
    B.cdz_set_profiling(h32, False)
    launches = int(tm[4])
    avg = tm[3]
    byt, flo = tensor_prop_algorithmic(sig, 9, 4)
    ach = byt / launches / (avg / 1e3) / 1e9
    out["roofline"] = {"kernel": "tz_prop<float>", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                       "traffic": measured_traffic("tensor", TENSOR_TRAFFIC_PROFILE),
                       "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                       "launches": launches, "avg_launch_ms": avg,
                       "algorithmic_bytes_per_launch": byt / launches,
                       "mfma_tflops": flo / (avg * launches / 1e3) / 1e12,
                       "mfma_frac": flo / (avg * launches / 1e3) / 1e12 / MFMA_FP32_PEAK_TFS,
                       "useful_flops_per_launch": flo / launches}
    return out


def extra_workloads(B, I):
    """The batch of 256 proteins (30..400 residues; forward + outside + 64 samples
    each, FP32; with direct launches and replayed hipGraphs), the 3900-nt instance (forward + outside, FP32 and FP64; 1000
    samples FP32) and its tensor-model free energy (FP32 and FP64), each timed once after one warm-up run, by HIP
    events."""
    out = {}
    probs = []
    for k in range(256):
        p, en4 = I.workload(4, index=k)
        probs.append(p)
    ns = np.array([p.n for p in probs])
    cells = float((ns * (ns + 1) // 2).sum())
    h = B.cdz_create(en4, "fp32")
    import ctypes
    for graphs in (1, 0):
        # hipGraphs (the launch-grouping tuner's trial runs capture their own
        # graphs; the timed run replays the settled one), then direct launches
        B.lib().cdz_debug_set_graphs(h.ptr, graphs)
        for rep in range(5 if graphs else 1):
            B.cdz_batch(h, probs, 64, I.sampler_seed(4), marginals=True)
        tm = B.cdz_last_timings(h)
        c, r = ctypes.c_int(0), ctypes.c_int(0)
        B.lib().cdz_debug_graph_counts(h.ptr, ctypes.byref(c), ctypes.byref(r))
        rec = {"dp_cells": cells, "ms_forward": tm[0], "ms_outside": tm[1], "ms_sample": tm[2],
               "dp_cells_per_s": cells / ((tm[0] + tm[1]) / 1e3), "dtype": "f32",
               "launches": "graph replay" if graphs else "direct", "graph_captures": c.value,
               "graph_replays": r.value}
        out["batch256_graphs" if graphs else "batch256"] = rec
        print(f"# batch256 {rec}", file=sys.stderr, flush=True)
    del h
    prob5, en5 = I.workload(5)
    n5 = prob5.n
    c5 = n5 * (n5 + 1) / 2
    for prec in ("fp32", "fp64"):
        h = B.cdz_create(en5, prec)
        for rep in range(2):
            B.cdz_reset(h)
            B.cdz_marginals(h, prob5)
        tm = B.cdz_last_timings(h)
        rec = {"dp_cells": c5, "ms_forward": tm[0], "ms_outside": tm[1],
               "dp_cells_per_s": c5 / ((tm[0] + tm[1]) / 1e3)}
        if prec == "fp32":
            B.cdz_sample(h, prob5, I.sampler_seed(5), N_SAMPLES)
            rec["ms_sample_1000"] = B.cdz_last_timings(h)[2]
        out[f"3900nt_{prec}"] = rec
        print(f"# 3900nt {prec} {rec}", file=sys.stderr, flush=True)
        del h
    # the tensor-model free energy of the 3900-nt protein (synthetic gamma 9 model)
    tprob, tmodel = I.tensor_workload(5)
    for prec in ("fp32", "fp64"):
        h = B.cdz_create(en5, prec)
        B.cdz_tensor_logz(h, tmodel, tprob)
        lz, _ = B.cdz_tensor_logz(h, tmodel, tprob)
        rec = {"ms": B.cdz_last_timings(h)[0], "logz": lz, "q_rows": int(9 * B.cdz_tensor_dims(tprob).sum())}
        out[f"tensor_3900nt_{prec}"] = rec
        print(f"# tensor 3900nt {prec} {rec}", file=sys.stderr, flush=True)
        del h
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true",
                    help="also time, once each, the 256-protein batch and the 3900-nt "
                         "instance (FP32 and FP64) and report them under extra_workloads")
    ap.add_argument("--no-mfe", dest="mfe", action="store_false",
                    help="skip timing the minimum free energy and its traceback on the same protein")
    ap.add_argument("--no-tensor", dest="tensor", action="store_false",
                    help="skip timing the tensor-model free energy (Sections 3b-3c) of the 900-nt protein")
    ap.add_argument("--tensor-steps", type=int, default=3,
                    help="timed tensor-model passes per precision (after one warm-up pass)")
    ap.add_argument("--no-freq", dest="freq", action="store_false",
                    help="skip timing frequency matching (Section S4e) on the same protein")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one device copy of 256 MiB first (the reference kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the per-instance dynamic program is measured on a "
              "single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    from paper_2604_19718_amd import binding as B
    from paper_2604_19718_amd import inputs as I

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prob, en = I.workload(3)
    n = prob.n
    cells = n * (n + 1) / 2
    seed = I.sampler_seed(3)
    h32 = B.cdz_create(en, "fp32")
    h64 = B.cdz_create(en, "fp64")

    for _ in range(args.warmup):
        run_step(B, h32, prob, seed)
    torch.cuda.synchronize()
    t_fwd, t_out, t_smp, walls = [], [], [], []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        run_step(B, h32, prob, seed)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        tm = B.cdz_last_timings(h32)
        t_fwd.append(tm[0])
        t_out.append(tm[1])
        t_smp.append(tm[2])
        print(f"# step fp32 wall {walls[-1]*1e3:.2f} ms fwd {tm[0]:.2f} out {tm[1]:.2f} "
              f"smp {tm[2]:.2f}", file=sys.stderr, flush=True)
    fwd = float(np.median(t_fwd))
    out = float(np.median(t_out))
    smp = float(np.median(t_smp))
    ms_fo = fwd + out
    value = cells / (ms_fo / 1e3)

    # full-FP64 GPU mode, same work
    f64 = []
    if args.fp64_steps > 0:
        run_step(B, h64, prob, seed)
    for _ in range(args.fp64_steps):
        run_step(B, h64, prob, seed)
        tm = B.cdz_last_timings(h64)
        f64.append(tm[0] + tm[1])
        print(f"# step fp64 fwd+out {f64[-1]:.2f} ms", file=sys.stderr, flush=True)
    ms_fo64 = float(np.median(f64)) if f64 else None

    # per-launch events around each diagonal launch; the dominant kernel (the
    # most time per step) is the outside diagonal kernel, the forward one is
    # reported beside it
    B.cdz_set_profiling(h32, True)
    run_step(B, h32, prob, seed)
    kt = B.cdz_kernel_timings(h32)
    B.cdz_set_profiling(h32, False)
    d = np.array([I.AA_DEGENERACY[ch] for ch in prob.prot for _ in range(3)], dtype=np.int64)
    bytes_out = algorithmic_bytes_out(d, 4)
    launches = int(kt[3])
    avg_ms = kt[2] / launches
    achieved = (bytes_out / launches) / (avg_ms / 1e3) / 1e9
    roof = {"kernel": "cdz_out_diag<float>", "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(), "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "launches": launches, "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": bytes_out / launches,
            "forward_kernel_ms": kt[0], "eta_kernel_ms": kt[4]}
    bytes_fwd = algorithmic_bytes_fwd(d, 4)
    fl = int(kt[1])
    fwd_avg = kt[0] / fl
    fwd_ach = (bytes_fwd / fl) / (fwd_avg / 1e3) / 1e9
    roof_fwd = {"kernel": "cdz_fwd_diag<float>", "bound": "hbm", "achieved": fwd_ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": fwd_ach / HBM_PEAK_GBS, "launches": fl, "avg_launch_ms": fwd_avg,
                "algorithmic_bytes_per_launch": bytes_fwd / fl}

    # frequency matching (Section S4e) on the same protein, FP32: target bonuses
    # those its codon weights were drawn from, r_tol 0.002, unlimited history
    freq = None
    if args.freq:
        ft = I.bonus_targets(I.config_seed(3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fb, ferr, fok = B.cdz_match_frequencies(h32, prob, ft, r_tol=0.002, max_eval=30, history=-1)
        torch.cuda.synchronize()
        fms = (time.perf_counter() - t0) * 1e3
        freq = {"evaluations": len(ferr), "converged": fok, "final_error": float(ferr[-1]),
                "r_tol": 0.002, "ms_total": fms, "ms_per_evaluation": fms / len(ferr),
                "errors": [float(e) for e in ferr]}
        print(f"# frequency matching {len(ferr)} evaluations {fms:.1f} ms", file=sys.stderr, flush=True)

    # minimum free energy with argmin traceback (Section 4d), FP64, same protein
    mfe = None
    if args.mfe:
        B.cdz_mfe(h64, prob)  # warm-up
        v_mfe, _, _ = B.cdz_mfe(h64, prob)
        tm = B.cdz_last_timings(h64)
        ops = algorithmic_ops_mfe(d)
        ach = ops / (tm[0] / 1e3) / 1e12
        # suboptimal states within 0.1 kT of the minimum (SI S4d), same protein, at most 500
        sub = B.cdz_subopt(h64, prob, 0.1, max_states=500)
        tms = B.cdz_last_timings(h64)
        subopt = {"gap_kT": 0.1, "states": int(len(sub[1])), "complete": bool(sub[4]), "ms_search": tms[2],
                  "ms_forward": tms[0]}
        print(f"# subopt gap 0.1: {len(sub[1])} states, search {tms[2]:.1f} ms", file=sys.stderr, flush=True)
        mfe = {"mfe_kT": v_mfe, "dtype": "f64", "ms_forward": tm[0], "ms_traceback": tm[2], "subopt": subopt,
               "roofline": {"kernel": "mfe_diag", "bound": "alu", "achieved": ach,
                            "peak": FP64_ALU_PEAK_TOPS, "unit": "TOP/s (FP64 add or min)",
                            "frac": ach / FP64_ALU_PEAK_TOPS, "ops": ops,
                            "note": "ops / forward time (fills, runs and exterior included)"}}
        print(f"# mfe {v_mfe:.4f} kT forward {tm[0]:.1f} ms traceback {tm[2]:.1f} ms", file=sys.stderr, flush=True)

    tensor = tensor_leg(B, I, h32, h64, max(1, args.tensor_steps)) if args.tensor else None

    res = {
        "metric": "DP cells/s + ms per forward+outside at 900 nt, FP32-scaled vs FP64, one GPU",
        "value": value, "unit": "DP cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": float(np.median(walls)) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one protein of 300 uniform random residues (900 nt), codon + "
                               "codon-pair weights, synthetic nearest-neighbour tables; forward + "
                               "outside marginals + 1000 samples per step",
                   "n_nt": n, "dp_cells": cells, "samples": N_SAMPLES},
        "ms_forward": fwd, "ms_outside": out, "ms_sample": smp, "ms_forward_outside": ms_fo,
        "ms_forward_outside_fp64": ms_fo64, "fp64_over_fp32": None if ms_fo64 is None else ms_fo64 / ms_fo,
        "roofline": roof,
        "roofline_forward": roof_fwd,
    }
    if freq is not None:
        res["frequency_matching"] = freq
    if mfe is not None:
        res["mfe"] = mfe
    if tensor is not None:
        res["tensor_model"] = tensor
    if args.extra:
        res["extra_workloads"] = extra_workloads(B, I)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(prob, en)
        if tensor is not None:
            tensor["cpu_baseline"] = tensor_cpu_baseline()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
