#!/usr/bin/env python3
"""Benchmark: the CCSD-like 4D contraction C[a,b,i,j] += sum_{c,k} A[a,c,i,k] * B[b,k,c,j]
(virtual extent 96 for a, b, c; occupied extent 32 for i, j, k; alpha = 1,
beta = 1; operands normal(0,1) * exp(-index gap / 8)) on one MI355X.

A step is one full contraction through the C ABI (plan cached, the GETT
kernel with its alpha/beta epilogue) with inputs resident in HBM.  The line
printed reports GFLOP/s of the FP64 matrix-core path as `value`, plus every
other compute mode that is built (GFLOP/s, MFMA-peak fraction and relative
error against the CPU FP64 oracle on sampled outputs), the roofline of the
dominant kernel timed with HIP events on its own stream, and the oracle
itself timed on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SPEC = "abij=acik*bkcj"
V, O = 96, 32
EXT = dict(a=V, b=V, c=V, i=O, j=O, k=O)
FLOPS = 2.0 * V ** 3 * O ** 3            # 2 * M * N * K, M = N = K = 3072
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6, "f16": 2516.6}
HBM_PEAK_GBS = 8000.0
# matrix-core products per algorithmic product, per compute mode
MODES = {
    "f64": dict(compute="f64", mfma="f64", products=1, tol=1e-12),
    "split_bf16": dict(compute="split_bf16", mfma="bf16", products=15, tol=1e-9),
    "split_bf16x3": dict(compute="split_bf16x3", mfma="bf16", products=6, tol=1e-5),
    "split_fp16x2": dict(compute="split_fp16x2", mfma="f16", products=3, tol=1e-5),
    "f32": dict(compute="default", mfma="f32", products=1, tol=1e-5, dtype="f32"),
}


def shape(labels):
    return tuple(EXT[c] for c in labels)


def make_inputs():
    import synth
    A = synth.decayed_normal(synth.config_seed(2, "A"), "acik", shape("acik"), "abc", "ijk")
    B = synth.decayed_normal(synth.config_seed(2, "B"), "bkcj", shape("bkcj"), "abc", "ijk")
    C0 = synth.decayed_normal(synth.config_seed(2, "C0"), "abij", shape("abij"), "abc", "ijk")
    return A, B, C0


def cpu_baseline(A, B, C0, seconds_target=15.0):
    """The oracle on the host cores over the first a-slabs of the output."""
    import oracle
    threads = oracle.max_threads()
    # calibrate on one a-slab, then size the sample to about seconds_target
    t0 = time.perf_counter()
    oracle.contract(SPEC, A[:1], B, C0[:1], alpha=1.0, beta=1.0)
    t1 = time.perf_counter() - t0
    slabs = int(max(1, min(V, seconds_target / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.contract(SPEC, A[:slabs], B, C0[:slabs], alpha=1.0, beta=1.0)
    dt = time.perf_counter() - t0
    flops = FLOPS * slabs / V
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "output slabs a < %d of %d (%.1f%% of config 2, FP64, beta=1), %.1f s" %
                      (slabs, V, 100.0 * slabs / V, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="all", help="comma list of compute modes, or all")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle
    import paper_2102_06827_amd as comet

    dev = torch.device("cuda:0")
    A, B, C0 = make_inputs()
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(11)
    pts = np.stack([rng.integers(0, n, 256) for n in shape("abij")], axis=1)
    ref_pts = oracle.contract_points(SPEC, A, B, pts, C0, alpha=1.0, beta=1.0)
    ref_pts32 = oracle.contract_points(SPEC, A.astype(np.float32), B.astype(np.float32), pts,
                                       C0.astype(np.float32), alpha=1.0, beta=1.0)

    results = {}
    want = list(MODES) if args.modes == "all" else args.modes.split(",")
    for name in want:
        cfg = MODES[name]
        tdt = torch.float32 if cfg.get("dtype") == "f32" else torch.float64
        Ad = torch.from_numpy(A).to(dev, tdt)
        Bd = torch.from_numpy(B).to(dev, tdt)
        C0d = torch.from_numpy(C0).to(dev, tdt)
        Cd = C0d.clone()
        try:
            comet.contract(SPEC, Ad, Bd, Cd, alpha=1.0, beta=1.0, compute=cfg["compute"])
        except comet.CometError as e:
            if e.name == "UNSUPPORTED":
                results[name] = {"status": "not built"}
                continue
            raise
        torch.cuda.synchronize()
        # accuracy of one result (beta = 1 on the original C0)
        idx = torch.from_numpy(pts).to(dev)
        got = Cd[tuple(idx.T)].double().cpu().numpy()
        err = oracle.relerr(got, ref_pts32 if cfg.get("dtype") == "f32" else ref_pts)
        for _ in range(args.warmup):
            comet.contract(SPEC, Ad, Bd, Cd, alpha=1.0, beta=1.0, compute=cfg["compute"])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            comet.contract(SPEC, Ad, Bd, Cd, alpha=1.0, beta=1.0, compute=cfg["compute"])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        gflops = FLOPS / (ms * 1e-3) / 1e9
        peak = PEAK_TFLOPS[cfg["mfma"]]
        results[name] = {
            "ms_per_step": round(ms, 4),
            "gflops": round(gflops, 1),
            "mfma_dtype": cfg["mfma"],
            "mfma_products": cfg["products"],
            "frac_mfma_peak": round(cfg["products"] * gflops / 1e3 / peak, 4),
            "relerr_vs_oracle": err,
            "tol": cfg["tol"],
            "within_tol": bool(err <= cfg["tol"]),
        }
        del Ad, Bd, C0d, Cd
        torch.cuda.empty_cache()

    head = results["f64"]
    ms = head["ms_per_step"]
    value = head["gflops"]
    achieved_tflops = FLOPS / (ms * 1e-3) / 1e12
    line = {
        "metric": "GFLOP/s & % MFMA peak per contraction: FP64 vs split-BF16x3 at stated rel err",
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "CCSD-like 4D contraction abij=acik*bkcj, V=96 O=32, alpha=1 beta=1, "
                               "decayed normal operands (M=N=K=3072)",
                   "spec": SPEC, "extents": EXT, "flops_per_step": FLOPS},
        "roofline": {"bound": "mfma", "achieved": round(achieved_tflops, 3), "peak": PEAK_TFLOPS["f64"],
                     "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_TFLOPS["f64"], 4),
                     "traffic": None, "kernel": "gett_kernel<double,double,128,128,16,K,N>"},
        "modes": results,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(A, B, C0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
