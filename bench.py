#!/usr/bin/env python3
"""Benchmark of the permuted tensor-contraction library on one MI355X.

Headline workload (the `value` of the printed line): the CCSD-like 4D
contraction C[a,b,i,j] += sum_{c,k} A[a,c,i,k] * B[b,k,c,j], virtual extent 96
(a, b, c), occupied extent 32 (i, j, k), alpha = 1, beta = 1, operands
normal(0,1) * exp(-index gap / 8).  A step is one full contraction through the
C ABI (plan cached) on the FP64 matrix cores, inputs resident in HBM.

The same line also carries, each timed with HIP events on the launch stream:
  modes      the headline contraction in every compute mode, with its relative
             error against the CPU FP64 oracle on sampled outputs;
  backward   forward + dA + dB of the same contraction (FP64, aligned BF16 and INT8 splits, BF16x3);
  triples    the 6D-output contraction C[a,b,c,i,j,k] = sum_d A[d,a,i,j] B[b,c,d,k]
             (virtual 32, occupied 16), bound by writing C to HBM;
  config1    the all-16 contraction (latency-bound): per call through the
             Python binding, and replayed from a HIP graph of plan executions
             (device time without host work); with the oracle's single-thread
             and all-core times;
  permute    the transpose kernel of the TTGT lowering on three shapes;
  ttgt_study every TTGT flattening of configs 2 and 3 timed, the planner's
             cost-model pick ranked among them, against GETT;
  chain      multi-operand chains of the paper's Table 1 shapes: the grouping
             with the fewest operations against the natural order;
  batch      1024 independent 4D contractions of six patterns with per-label
             extents from {8,...,64}, forward + backward in one persistent
             launch replayed from a HIP graph (FP32 and BF16x3);
  batch_labels  contractions with a label in C, A and B (batched products),
             against torch.bmm where the layout allows;
  roofline   of the headline kernel; cpu_baseline: the oracle on the host.

Before each timed region the workload runs untimed for a quarter of a second
(on top of the warm-up steps), so that every figure is taken at the clocks
the GPU sustains under load rather than during their ramp from idle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SPEC = "abij=acik*bkcj"
V, O = 96, 32
EXT = dict(a=V, b=V, c=V, i=O, j=O, k=O)
FLOPS = 2.0 * V ** 3 * O ** 3            # 2 * M * N * K, M = N = K = 3072
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6, "f16": 2516.6, "i8": 5033.2}
HBM_PEAK_GBS = 8000.0
# The headline contraction runs as one launch group of the gather kernel:
# the whole output tiles and the summation pieces of the tiles left after
# the last full round in one launch (gett_whole_piece_kernel; gett_kernel
# and gett_sk_kernel when stream-K is planned instead), then the sum of
# those pieces (gett_piece_fixup_kernel or gett_fixup_kernel).  HBM bytes of one group from FETCH_SIZE / WRITE_SIZE
# counters scaled by a plain 1 GiB copy (profiles/gett_f64_ccsd_v96_o32_hbm_counters.md);
# valid only for the schedule and kernel version recorded, null otherwise.
HEADLINE_TRAFFIC = {"schedule": {"tile": 3, "sk_tiles": 64, "sk_blocks": 512, "even": 1}, "kernel_version": "k11",
                    "bytes": 971436304}
KERNEL_VERSION = "k11"


def headline_kernels(d):
    # the headline's output is whole 128 x 128 tiles over whole K steps: tile
    # 3 runs its unmasked variant (last template argument true)
    t = d["tile"]
    full = ", true" if t == 3 else ""
    if d.get("sk_tiles") and d.get("even"):
        return ["gett_whole_piece_kernel<double, double, %d, 0, 1, true, true%s>" % (t, full),
                "gett_piece_fixup_kernel<double, double, %d>" % t]
    ks = ["gett_kernel<double, double, %d, 0, 1, true, true%s>" % (t, full)]
    if d.get("sk_tiles"):
        ks += ["gett_sk_kernel<double, double, %d, 0, 1, true, true>" % t, "gett_fixup_kernel<double, double, %d>" % t]
    return ks
MODES = {
    "f64": dict(compute="f64", mfma="f64", products=1, tol=1e-12),
    "split_bf16": dict(compute="split_bf16", mfma="bf16", products=15, tol=1e-9),
    "split_bf16x3": dict(compute="split_bf16x3", mfma="bf16", products=6, tol=1e-5),
    "split_fp16x2": dict(compute="split_fp16x2", mfma="f16", products=3, tol=1e-5),
    "split_int8": dict(compute="split_int8", mfma="i8", products=21, tol=1e-9),
    "f32": dict(compute="default", mfma="f32", products=1, tol=1e-5, dtype="f32"),
    # the TTGT lowering of Section 2 (permute A, B, C around one matrix product)
    "f64_ttgt": dict(compute="f64", mfma="f64", products=1, tol=1e-12, path="ttgt"),
}


def shape(labels, ext=EXT):
    return tuple(ext[c] for c in labels)


def split_spec(spec):
    """(C, A, B) label strings of "C=A*B"."""
    s = "".join(spec.split())
    c, ab = s.split("=")
    a, b = ab.split("*")
    return c, a, b


def grad_specs(spec):
    """The contractions giving dA and dB from dC: "<A>=<C>*<B>", "<B>=<A>*<C>"."""
    c, a, b = split_spec(spec)
    return "%s=%s*%s" % (a, c, b), "%s=%s*%s" % (b, a, c)


def relerr(got, ref):
    """Relative Frobenius error, accumulated in long double."""
    g = np.asarray(got, dtype=np.longdouble).ravel()
    r = np.asarray(ref, dtype=np.longdouble).ravel()
    den = np.sqrt(np.sum(r * r))
    num = np.sqrt(np.sum((g - r) * (g - r)))
    return float(num / den) if den > 0 else float(num)


# Accuracy checks are recorded by the GPU sections (inputs, sample points, the
# GPU's values at them) and evaluated against the CPU FP64 oracle in the CPU
# leg at the end (cpu_leg), which also times the oracle.  Each check names the
# field of the output line its error goes to.
CHECKS = []


def check_points(where, spec, A, B, pts, got, C0=None, alpha=1.0, beta=0.0, tol=None):
    CHECKS.append(dict(kind="points", where=where, spec=spec, A=A, B=B, C0=C0, alpha=alpha, beta=beta, pts=pts,
                       got=got, tol=tol))


def check_full(where, spec, A, B, got, W=None, dA=None, dB=None):
    CHECKS.append(dict(kind="full", where=where, spec=spec, A=A, B=B, got=got, W=W, dA=dA, dB=dB))


def set_field(line, where, value):
    d = line
    for k in where[:-1]:
        d = d[k]
    d[where[-1]] = value


def make_inputs():
    import synth
    A = synth.decayed_normal(synth.config_seed(2, "A"), "acik", shape("acik"), "abc", "ijk")
    B = synth.decayed_normal(synth.config_seed(2, "B"), "bkcj", shape("bkcj"), "abc", "ijk")
    C0 = synth.decayed_normal(synth.config_seed(2, "C0"), "abij", shape("abij"), "abc", "ijk")
    return A, B, C0


def prime(fn, seconds=0.25):
    """Run fn untimed for about `seconds`, synchronizing every few calls, so
    that the timed runs that follow start at the sustained clocks: on MI355X
    a kernel sequence started from idle takes some 25 ms of load to get
    there (the headline gather kernel ramps from about 1.0 to 0.82 ms per
    call), and host work between sections lets the clocks drop again."""
    import torch
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def timed(fn, reps, stream):
    """Mean milliseconds of fn() over reps runs, HIP events on `stream`."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_leg(line, A, B, C0, seconds_target=15.0):
    """The CPU FP64 oracle: evaluate every recorded accuracy check, then time
    it on the host cores over the first a-slabs of the headline output."""
    import oracle
    for ch in CHECKS:
        if ch["kind"] == "points":
            ref = oracle.contract_points(ch["spec"], ch["A"], ch["B"], ch["pts"], ch["C0"], alpha=ch["alpha"],
                                         beta=ch["beta"])
            err = relerr(ch["got"], ref)
            prev = line
            for k in ch["where"][:-1]:
                prev = prev[k]
            # several checks may report into one field: keep the largest error
            err = max(err, prev.get(ch["where"][-1]) or 0.0)
            set_field(line, ch["where"], err)
            if ch["tol"] is not None:
                set_field(line, ch["where"][:-1] + ["within_tol"], bool(err <= ch["tol"]))
        else:
            errs = [relerr(ch["got"], oracle.contract(ch["spec"], ch["A"], ch["B"]))]
            if ch["W"] is not None:
                gA, gB, _ = oracle.grad(ch["spec"], ch["A"], ch["B"], ch["W"])
                errs += [relerr(ch["dA"], gA), relerr(ch["dB"], gB)]
            prev = line
            for k in ch["where"][:-1]:
                prev = prev[k]
            prev[ch["where"][-1]] = max([prev.get(ch["where"][-1]) or 0.0] + errs)
    threads = oracle.max_threads()
    c1 = line.get("config1")
    if c1 is not None:
        spec, _ = CONFIG1
        for key, nt in (("oracle_ms_all_cores", threads), ("oracle_ms_1thread", 1)):
            t0 = time.perf_counter()
            oracle.contract(spec, c1["A"], c1["B"], nthreads=nt)
            c1[key] = round((time.perf_counter() - t0) * 1e3, 3)
        oracle.contract(spec, c1["A"][:1], c1["B"], nthreads=threads)   # restore the thread count
    line["cpu_baseline"] = cpu_baseline(oracle, A, B, C0, seconds_target)


def cpu_baseline(oracle, A, B, C0, seconds_target=15.0):
    """The oracle on the host cores over the first a-slabs of the output."""
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.contract(SPEC, A[:1], B, C0[:1], alpha=1.0, beta=1.0, nthreads=threads)
    t1 = time.perf_counter() - t0
    slabs = int(max(1, min(V, seconds_target / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.contract(SPEC, A[:slabs], B, C0[:slabs], alpha=1.0, beta=1.0, nthreads=threads)
    dt = time.perf_counter() - t0
    flops = FLOPS * slabs / V
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": "output slabs a < %d of %d (%.1f%% of the headline contraction, FP64, beta=1), %.1f s" %
                      (slabs, V, 100.0 * slabs / V, dt)}


def cpu_model():
    """The host CPU's model name as lscpu reports it (/proc/cpuinfo if lscpu is absent)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_modes(comet, A, B, C0, steps, warmup, want):
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(11)
    pts = np.stack([rng.integers(0, n, 256) for n in shape("abij")], axis=1)
    results = {}
    for name in want:
        cfg = MODES[name]
        tdt = torch.float32 if cfg.get("dtype") == "f32" else torch.float64
        Ad, Bd = torch.from_numpy(A).to(dev, tdt), torch.from_numpy(B).to(dev, tdt)
        Cd = torch.from_numpy(C0).to(dev, tdt)
        if cfg.get("path"):
            plan = comet.Plan(SPEC, Ad, Bd, Cd, compute=cfg["compute"], path=cfg["path"])
            run = lambda: plan(Ad, Bd, Cd, alpha=1.0, beta=1.0)
        else:
            run = lambda: comet.contract(SPEC, Ad, Bd, Cd, alpha=1.0, beta=1.0, compute=cfg["compute"])
        run()
        torch.cuda.synchronize()
        idx = torch.from_numpy(pts).to(dev)
        got = Cd[tuple(idx.T)].double().cpu().numpy()
        if cfg.get("dtype") == "f32":
            check_points(["modes", name, "relerr_vs_oracle"], SPEC, A.astype(np.float32), B.astype(np.float32), pts,
                         got, C0.astype(np.float32), 1.0, 1.0, cfg["tol"])
        else:
            check_points(["modes", name, "relerr_vs_oracle"], SPEC, A, B, pts, got, C0, 1.0, 1.0, cfg["tol"])
        prime(run)
        for _ in range(warmup):
            run()
        ms = timed(run, steps, stream)
        gflops = FLOPS / (ms * 1e-3) / 1e9
        results[name] = {
            "ms": round(ms, 4), "gflops": round(gflops, 1), "mfma_dtype": cfg["mfma"],
            "mfma_products": cfg["products"],
            "frac_mfma_peak": round(cfg["products"] * gflops / 1e3 / PEAK_TFLOPS[cfg["mfma"]], 4),
            "relerr_vs_oracle": None, "tol": cfg["tol"], "within_tol": None,
        }
        del Ad, Bd, Cd
        torch.cuda.empty_cache()
    return results


def bench_backward(comet, A, B, C0, reps):
    """forward + dA + dB for loss = sum(C * W): FP64, the aligned BF16 and INT8 splits and BF16x3."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    W = synth.uniform(synth.config_seed(4, "W"), shape("abij"))
    sa, sb = grad_specs(SPEC)
    rng = np.random.default_rng(12)
    ptsA = np.stack([rng.integers(0, n, 128) for n in shape("acik")], axis=1)
    ptsB = np.stack([rng.integers(0, n, 128) for n in shape("bkcj")], axis=1)
    out = {}
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    Wd = torch.from_numpy(W).to(dev)
    C = torch.empty(shape("abij"), dtype=torch.float64, device=dev)
    dA = torch.empty_like(Ad)
    dB = torch.empty_like(Bd)
    for mode in ("f64", "split_bf16", "split_int8", "split_bf16x3"):
        def step():
            comet.contract(SPEC, Ad, Bd, C, compute=mode)
            comet.contract(sa, Wd, Bd, dA, compute=mode)
            comet.contract(sb, Ad, Wd, dB, compute=mode)
        step()
        torch.cuda.synchronize()
        check_points(["backward", mode, "relerr_dA"], sa, W, B, ptsA,
                     dA[tuple(torch.from_numpy(ptsA).to(dev).T)].cpu().numpy())
        check_points(["backward", mode, "relerr_dB"], sb, A, W, ptsB,
                     dB[tuple(torch.from_numpy(ptsB).to(dev).T)].cpu().numpy())
        prime(step)
        ms = timed(step, reps, stream)
        out[mode] = {"ms": round(ms, 4), "gflops": round(3 * FLOPS / (ms * 1e-3) / 1e9, 1),
                     "relerr_dA": None, "relerr_dB": None}
    return out


def bench_triples(comet, reps):
    """C[a,b,c,i,j,k] = sum_d A[d,a,i,j] * B[b,c,d,k]: writing C (1.07 GB) dominates."""
    import torch
    import synth
    ext = dict(a=32, b=32, c=32, d=32, i=16, j=16, k=16)
    spec = "abcijk=daij*bcdk"
    A = synth.uniform(synth.config_seed(3, "A"), shape("daij", ext))
    B = synth.uniform(synth.config_seed(3, "B"), shape("bcdk", ext))
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    C = torch.empty(shape("abcijk", ext), dtype=torch.float64, device=dev)
    flops = 2.0 * 32 ** 4 * 16 ** 3
    nbytes = 8.0 * (A.size + B.size + C.numel())
    rng = np.random.default_rng(13)
    pts = np.stack([rng.integers(0, n, 256) for n in C.shape], axis=1)
    flush = torch.ones(512 * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
    out = {}
    for mode in ("f64", "split_bf16", "split_bf16x3", "split_fp16x2", "split_int8", "f64_ttgt", "f64_whole_tiles"):
        if mode == "f64_ttgt":
            plan = comet.Plan(spec, Ad, Bd, C, compute="f64", path="ttgt")
            run = lambda: plan(Ad, Bd, C)
        elif mode == "f64_whole_tiles":
            # the gather kernel with a workgroup per tile, for comparison with
            # the short-summation kernel the planner takes
            os.environ["COMET_GETT_SHORTK"] = "0"
            try:
                plan = comet.Plan(spec, Ad, Bd, C, compute="f64")
            finally:
                os.environ.pop("COMET_GETT_SHORTK", None)
            run = lambda: plan(Ad, Bd, C)
        else:
            run = lambda: comet.contract(spec, Ad, Bd, C, compute=mode)
        run()
        torch.cuda.synchronize()
        check_points(["triples", mode, "relerr_vs_oracle"], spec, A, B, pts,
                     C[tuple(torch.from_numpy(pts).to(dev).T)].cpu().numpy())
        prime(run)
        tot = 0.0
        for _ in range(reps):
            # evict the 256 MB last-level cache between runs by reading 512 MB:
            # a write would leave it full of dirty lines whose write-back the
            # timed run would pay for
            flush.sum()
            tot += timed(run, 1, stream)
        ms = tot / reps
        out[mode] = {"ms": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                     "hbm_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm_peak": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "relerr_vs_oracle": None}
        if mode == "f64":
            d = comet.Plan(spec, Ad, Bd, C, compute="f64").describe()
            out[mode]["schedule"] = {k: d[k] for k in ("path", "tile", "shortk", "sk_tiles")}
    del C, flush
    torch.cuda.empty_cache()
    return out


CONFIG1 = ("abij=acik*cbkj", dict(a=16, b=16, c=16, i=16, j=16, k=16))


def bench_config1(comet, reps=50):
    """Config 1 (all extents 16, FP64, beta = 0): latency-bound, one launch."""
    import torch
    import synth
    spec, ext = CONFIG1
    c, a, b = split_spec(spec)
    A = synth.uniform(synth.config_seed(1, "A"), shape(a, ext))
    B = synth.uniform(synth.config_seed(1, "B"), shape(b, ext))
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = comet.contract(spec, Ad, Bd)
    torch.cuda.synchronize()
    check_full(["config1", "relerr_vs_oracle"], spec, A, B, C.cpu().numpy())
    ms = timed(lambda: comet.contract(spec, Ad, Bd, C), reps, torch.cuda.current_stream())
    flops = 2.0 * 16 ** 6
    # the same contraction through a plan captured in a HIP graph: the device
    # time per contraction without the per-call host work
    plan = comet.Plan(spec, Ad, Bd, C, compute="f64")
    ws = plan.workspace(Ad.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan(Ad, Bd, C, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(10):
            plan(Ad, Bd, C, workspace=ws)
    graph.replay()
    torch.cuda.synchronize()
    graph_ms = timed(graph.replay, max(1, reps // 10), torch.cuda.current_stream()) / 10
    return {"ms": round(ms, 5), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
            "graph_ms": round(graph_ms, 5), "graph_gflops": round(flops / (graph_ms * 1e-3) / 1e9, 1),
            "relerr_vs_oracle": None, "oracle_ms_1thread": None, "oracle_ms_all_cores": None, "A": A, "B": B}


def bench_chain(comet, reps=5):
    """Multi-operand chains (Section 6; the shapes of the paper's Table 1) at
    NWChem-like extents (occupied 32, virtual 96): the planner's grouping
    against the natural left-to-right order, both on the GPU, FP64."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    O_, V_ = 32, 96
    out = {}
    g = torch.Generator(device=dev)
    g.manual_seed(17)
    for rhs in ("cdmn*inad*mc", "cdmn*id*na*mc", "mnef*am*fn*ebij"):
        ops = rhs.split("*")
        once = [l for l in dict.fromkeys("".join(ops)) if sum(l in o for o in ops) == 1]
        spec = "".join(once) + "=" + rhs
        ext = {l: (O_ if l in "ijmn" else V_) for l in set(rhs) - {"*"}}
        ts = [torch.rand(tuple(ext[l] for l in o), dtype=torch.float64, device=dev, generator=g) for o in ops]
        plan = comet.chain_plan(spec, ext)
        res = comet.contract_chain(spec, ts)
        t_best = timed(lambda: comet.contract_chain(spec, ts, res), reps, stream)

        def natural():
            acc, lab = ts[0], ops[0]
            for i in range(1, len(ops)):
                rest = set(once).union(*[set(o) for o in ops[i + 1:]])
                keep = "".join(once) if i == len(ops) - 1 else \
                    "".join(l for l in dict.fromkeys(lab + ops[i]) if l in rest)
                acc = comet.contract("%s=%s*%s" % (keep, lab, ops[i]), acc, ts[i])
                lab = keep
            return acc
        nat = natural()
        torch.cuda.synchronize()
        err = float(((nat - res).norm() / res.norm()).item())
        t_nat = timed(natural, 1, stream)
        out[spec] = {"flops": plan["flops"], "natural_flops": plan["natural_flops"],
                     "order": [st["spec"] for st in plan["steps"]], "ms": round(t_best, 4),
                     "natural_ms": round(t_nat, 4), "speedup": round(t_nat / t_best, 1),
                     "relerr_vs_natural": err}
        del ts, res, nat
        torch.cuda.empty_cache()
    return out


def bench_permute(comet, reps):
    """The permute kernel (TTGT's transposes and ta.copy): HBM bytes moved per second.

    Cases: a config-2 operand brought into (M, K) order, the config-3 output
    returned from (M, N) order to its own (both share a short unit dimension),
    and a plain 8192 x 8192 transpose."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    flush = torch.ones(512 * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
    cases = [("aick=acik", dict(a=96, c=96, i=32, k=32)),
             ("abcijk=aijbck", dict(a=32, b=32, c=32, i=16, j=16, k=16)),
             ("ji=ij", dict(i=8192, j=8192))]
    out = {}
    g = torch.Generator(device=dev)
    g.manual_seed(15)
    for spec, ext in cases:
        lo, li = spec.split("=")
        x = torch.rand(tuple(ext[c] for c in li), dtype=torch.float64, device=dev, generator=g)
        y = torch.empty(tuple(ext[c] for c in lo), dtype=torch.float64, device=dev)
        comet.permute(spec, x, y)
        torch.cuda.synchronize()
        exact = bool(torch.equal(y, x.permute(*[li.index(c) for c in lo])))
        tot = 0.0
        for _ in range(reps):
            flush.sum()          # clean cold cache, as for the triples contraction
            tot += timed(lambda: comet.permute(spec, x, y), 1, stream)
        ms = tot / reps
        nbytes = 2.0 * x.numel() * 8
        out[spec] = {"ms": round(ms, 4), "bytes": nbytes, "hbm_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm_peak": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "exact": exact}
        del x, y
    del flush
    torch.cuda.empty_cache()
    return out


def bench_ttgt_study(comet, reps=10):
    """TTGT permutation choice on MI355X (Section 6): time every valid
    flattening -- each order of the M, N and K label groups, each operand
    stored K-major or not -- and rank the planner's pick (the MI355X time
    model), the published position weights' pick and the autotuner's pick
    among them, against GETT too.  Config 2 (FP64) and config 3 (FP64,
    beta = 0)."""
    import itertools
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    cases = [("config2", SPEC, EXT, 1.0), ("config3", "abcijk=daij*bcdk",
                                           dict(a=32, b=32, c=32, d=32, i=16, j=16, k=16), 0.0)]
    g = torch.Generator(device=dev)
    g.manual_seed(16)
    for name, spec, ext, beta in cases:
        c, a, b = split_spec(spec)
        A = torch.rand(shape(a, ext), dtype=torch.float64, device=dev, generator=g)
        B = torch.rand(shape(b, ext), dtype=torch.float64, device=dev, generator=g)
        C0 = torch.rand(shape(c, ext), dtype=torch.float64, device=dev, generator=g)
        C = torch.empty_like(C0)
        ref = comet.Plan(spec, A, B, C, compute="f64", path="gett")
        C.copy_(C0)
        ref(A, B, C, beta=beta)
        torch.cuda.synchronize()
        R = C.clone()
        prime(lambda: ref(A, B, C, beta=beta))
        t_gett = timed(lambda: ref(A, B, C, beta=beta), reps, stream)
        M = [l for l in a if l in c]
        N = [l for l in b if l in c]
        K = [l for l in a if l not in c]
        pick = comet.analyze(spec, [ext[l] for l in spec_labels(spec)], path="ttgt")["ttgt"]
        pick_key = (pick["A"], pick["B"], pick["C"])
        # the published position weights' pick, for comparison
        os.environ["COMET_TTGT_MODEL"] = "weights"
        try:
            wpick = comet.analyze(spec, [ext[l] for l in spec_labels(spec)], path="ttgt")["ttgt"]
        finally:
            os.environ.pop("COMET_TTGT_MODEL", None)
        wpick_key = (wpick["A"], wpick["B"], wpick["C"])
        rows = []
        for mo in itertools.permutations(M):
            for no in itertools.permutations(N):
                for ko in itertools.permutations(K):
                    mo_, no_, ko_ = "".join(mo), "".join(no), "".join(ko)
                    for swap in (0, 1):
                        for la in (0, 1):
                            for lb in (0, 1):
                                r_, c_ = (no_, mo_) if swap else (mo_, no_)
                                left = ko_ + r_ if la else r_ + ko_
                                right = c_ + ko_ if lb else ko_ + c_
                                ap, bp = (right, left) if swap else (left, right)
                                rows.append((ap, bp, r_ + c_))
        rows = sorted(set(rows))
        times = {}
        worst_err = 0.0
        for ap, bp, cp in rows:
            os.environ["COMET_TTGT_ORDER"] = "%s|%s|%s" % (ap, bp, cp)
            try:
                plan = comet.Plan(spec, A, B, C, compute="f64", path="ttgt")
            finally:
                os.environ.pop("COMET_TTGT_ORDER", None)
            C.copy_(C0)
            plan(A, B, C, beta=beta)
            torch.cuda.synchronize()
            err = float(((C - R).norm() / R.norm()).item())
            worst_err = max(worst_err, err)
            # two untimed runs first: a new plan's first calls also pay for
            # its workspace's first touch
            timed(lambda: plan(A, B, C, beta=beta), 2, stream)
            times[(ap, bp, cp)] = timed(lambda: plan(A, B, C, beta=beta), reps, stream)
            del plan
        ranked = sorted(times, key=times.get)
        best = ranked[0]
        # the flattening the autotuner picks when TTGT is asked for (it times
        # every one in its own runs), ranked by this study's timings
        with tempfile.TemporaryDirectory() as td:
            comet.autotune(os.path.join(td, "tune.json"), 2)
            try:
                tuned = comet.Plan(spec, A, B, C, compute="f64", path="ttgt").describe()["ttgt"]
            finally:
                comet.autotune(None, 0)
        tuned_key = (tuned["A"], tuned["B"], tuned["C"])
        out[name] = {"candidates": len(rows), "gett_ms": round(t_gett, 4),
                     "best_ttgt": {"orders": "|".join(best), "ms": round(times[best], 4)},
                     "planner_pick": {"orders": "|".join(pick_key), "ms": round(times.get(pick_key, float("nan")), 4),
                                      "rank": ranked.index(pick_key) + 1 if pick_key in times else None,
                                      "model_us": round(pick["model_us"], 1)},
                     "weights_pick": {"orders": "|".join(wpick_key), "ms": round(times.get(wpick_key, float("nan")), 4),
                                      "rank": ranked.index(wpick_key) + 1 if wpick_key in times else None,
                                      "cost": wpick["cost"]},
                     "tuned_pick": {"orders": "|".join(tuned_key), "ms": round(times.get(tuned_key, float("nan")), 4),
                                    "rank": ranked.index(tuned_key) + 1 if tuned_key in times else None},
                     "worst_ttgt": {"orders": "|".join(ranked[-1]), "ms": round(times[ranked[-1]], 4)},
                     "max_relerr_vs_gett": worst_err}
        del A, B, C, C0, R, ref
        torch.cuda.empty_cache()
    return out


def spec_labels(spec):
    """Distinct labels in order of first appearance scanning C, A, B."""
    seen = []
    for ch in spec.replace("=", "").replace("*", ""):
        if ch not in seen:
            seen.append(ch)
    return seen


def bench_batch(comet, reps, n=1024):
    """1024 contractions, forward + dA + dB, one persistent launch in a HIP graph."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    probs = synth.batch_problems(n, synth.config_seed(5, "A"))
    f = torch.float32
    tensors, problems = [], []
    flops = 0.0
    for i, (spec, ext) in enumerate(probs):
        c, a, b = split_spec(spec)
        A = synth.uniform_torch(5_000_000 + 10 * i + 1, shape(a, ext), f, dev)
        B = synth.uniform_torch(5_000_000 + 10 * i + 2, shape(b, ext), f, dev)
        W = synth.uniform_torch(5_000_000 + 10 * i + 4, shape(c, ext), f, dev)
        C = torch.empty(shape(c, ext), dtype=f, device=dev)
        dA = torch.empty_like(A)
        dB = torch.empty_like(B)
        sa, sb = grad_specs(spec)
        problems += [dict(spec=spec, A=A, B=B, C=C), dict(spec=sa, A=W, B=B, C=dA),
                     dict(spec=sb, A=A, B=W, C=dB)]
        tensors.append((spec, A, B, W, C, dA, dB))
        prod = 1
        for v in ext.values():
            prod *= v
        flops += 3 * 2.0 * prod
    out = {"problems": n, "contractions": 3 * n, "flops_per_step": flops,
           "autotune": os.environ.get("COMET_AUTOTUNE", "off")}
    ws = torch.empty(256, dtype=torch.uint8, device=dev)
    # oracle check: every contraction of the seeded sample (128 problems,
    # every problem of at most 2^24 FLOPs and the 20 heaviest) at 64 output
    # points each, corners included; the oracle evaluates them in the CPU leg
    sample = synth.batch_check_sample(probs)
    host = {}
    for i in sample:
        spec, A, B, W = tensors[i][:4]
        host[i] = (A.cpu().numpy(), B.cpu().numpy(), W.cpu().numpy())

    def points(shp, seed):
        rng = np.random.default_rng(seed)
        pts = np.stack([rng.integers(0, e, 62) for e in shp], axis=1).reshape(62, len(shp))
        return np.concatenate([np.zeros((1, len(shp)), np.int64), np.array([shp], np.int64) - 1, pts])

    for mode in ("default", "split_bf16x3"):
        key = "f32" if mode == "default" else "split_bf16x3"
        batch = comet.Batch(problems, dtype=f, compute=mode)
        desc = batch.describe()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            batch(workspace=ws)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            batch(workspace=ws)
        g.replay()
        torch.cuda.synchronize()
        prime(g.replay)
        ms = timed(g.replay, reps, torch.cuda.current_stream())
        gflops = flops / (ms * 1e-3) / 1e9
        mf = "f32" if mode == "default" else "bf16"
        prods = 1 if mode == "default" else 6
        out[key] = {
            "ms": round(ms, 3), "gflops": round(gflops, 1),
            "frac_mfma_peak": round(prods * gflops / 1e3 / PEAK_TFLOPS[mf], 4),
            "max_relerr_sampled": None, "sampled_problems": len(sample), "points_per_contraction": 64,
            "tiles": desc["tiles"], "problems_per_class": desc["classes"], "operand_copies": desc["copies"],
            "tuned_problems": desc["tuned"]}
        for i in sample:
            spec, A, B, W, C, dA, dB = tensors[i]
            An, Bn, Wn = host[i]
            c, a, b = split_spec(spec)
            sa, sb = grad_specs(spec)
            for sp, X, Y, got in ((spec, An, Bn, C), (sa, Wn, Bn, dA), (sb, An, Wn, dB)):
                pts = points(tuple(got.shape), 7000 + i)
                vals = got[tuple(torch.from_numpy(pts.T).to(got.device))].double().cpu().numpy()
                check_points(["batch", key, "max_relerr_sampled"], sp, X, Y, pts, vals)
        del g, batch
    del tensors, problems
    torch.cuda.empty_cache()
    return out


# Batch labels (one label in C, A and B): batched matrix products with one
# tiles x entries launch, FP64.
BATCH_LABEL_CASES = [
    ("bij=bik*bkj", dict(b=64, i=512, j=512, k=512)),      # a few large entries
    ("bij=bik*bkj", dict(b=4096, i=64, j=64, k=64)),       # many small entries
    ("ibj=kbi*jbk", dict(b=32, i=384, j=384, k=384)),      # batch label inside every tensor
]


def bench_batch_labels(comet, reps=5):
    """Contractions with a batch label (FP64), against torch.bmm on the same
    data where the layout is a plain batched product; sampled outputs are
    checked against the oracle in the CPU leg."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    g = torch.Generator(device=dev)
    g.manual_seed(19)
    rng = np.random.default_rng(19)
    for n, (spec, ext) in enumerate(BATCH_LABEL_CASES):
        c, a, b = split_spec(spec)
        A = torch.rand(shape(a, ext), dtype=torch.float64, device=dev, generator=g) * 2 - 1
        B = torch.rand(shape(b, ext), dtype=torch.float64, device=dev, generator=g) * 2 - 1
        C = comet.contract(spec, A, B)
        torch.cuda.synchronize()
        pts = np.stack([rng.integers(0, e, 128) for e in shape(c, ext)], axis=1)
        got = C[tuple(torch.from_numpy(pts[:, d]).to(dev) for d in range(len(c)))].cpu().numpy()
        key = "%s %s" % (spec, ",".join("%s=%d" % kv for kv in ext.items()))
        check_points(["batch_labels", key, "relerr_vs_oracle"], spec, A.cpu().numpy(), B.cpu().numpy(), pts, got,
                     tol=1e-12)
        comet.contract(spec, A, B, C)
        ms = timed(lambda: comet.contract(spec, A, B, C), reps, stream)
        flops = 2.0 * float(np.prod(list(ext.values())))
        d = comet.Plan(spec, A, B, C).describe()
        rec = {"ms": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
               "frac_mfma_peak": round(flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["f64"], 4),
               "tile": d["tile"], "relerr_vs_oracle": None}
        if spec == "bij=bik*bkj":
            R = torch.bmm(A, B)
            rec["max_abs_diff_vs_torch_bmm"] = float((R - C).abs().max().item())
            t = timed(lambda: torch.bmm(A, B, out=R), reps, stream)
            rec["torch_bmm_ms"] = round(t, 4)
            rec["torch_bmm_gflops"] = round(flops / (t * 1e-3) / 1e9, 1)
            del R
        out[key] = rec
        del A, B, C
        torch.cuda.empty_cache()
    return out


def profile_pass(comet, which):
    """Each workload a few times, untimed, for a profiler's kernel-trace or
    counter pass (the counters of a kernel do not depend on the operand
    values, so the batched workload takes plain random values).  About one
    second of headline products first brings the clocks up, so that the
    trace's durations are those of the timed runs."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    A, B, C0 = make_inputs()
    Ad, Bd, Cd = (torch.from_numpy(x).to(dev) for x in (A, B, C0))
    p = comet.Plan(SPEC, Ad, Bd, Cd, compute="f64")
    t_end = time.perf_counter() + 1.0
    while time.perf_counter() < t_end:
        p(Ad, Bd, Cd, beta=1.0)
        torch.cuda.synchronize()
    print("warm-up done", flush=True)
    if "headline" in which or "split" in which:
        if "headline" in which:
            for _ in range(10):
                p(Ad, Bd, Cd, beta=1.0)
            torch.cuda.synchronize()
            print("headline done", flush=True)
        if "split" in which:
            for mode in ("split_bf16", "split_int8", "split_bf16x3", "split_fp16x2", "f32"):
                if mode == "f32":
                    A32, B32, C32 = Ad.float(), Bd.float(), Cd.float()
                    p = comet.Plan(SPEC, A32, B32, C32)
                    for _ in range(3):
                        p(A32, B32, C32, beta=1.0)
                else:
                    p = comet.Plan(SPEC, Ad, Bd, Cd, compute=mode)
                    for _ in range(3):
                        p(Ad, Bd, Cd, beta=1.0)
                torch.cuda.synchronize()
                print(mode, "done", flush=True)
    if "triples" in which:
        A = torch.rand((32, 32, 16, 16), dtype=torch.float64, device=dev)
        B = torch.rand((32, 32, 32, 16), dtype=torch.float64, device=dev)
        C = torch.empty((32, 32, 32, 16, 16, 16), dtype=torch.float64, device=dev)
        p = comet.Plan("abcijk=daij*bcdk", A, B, C)
        for _ in range(10):
            p(A, B, C)
        torch.cuda.synchronize()
        print("triples done", flush=True)
    if "batch" in which:
        f = torch.float32
        problems = []
        for i, (spec, ext) in enumerate(synth.batch_problems(1024, synth.config_seed(5, "A"))):
            c, a, b = split_spec(spec)
            A = torch.rand(shape(a, ext), dtype=f, device=dev)
            B = torch.rand(shape(b, ext), dtype=f, device=dev)
            W = torch.rand(shape(c, ext), dtype=f, device=dev)
            sa, sb = grad_specs(spec)
            problems += [dict(spec=spec, A=A, B=B, C=torch.empty(shape(c, ext), dtype=f, device=dev)),
                         dict(spec=sa, A=W, B=B, C=torch.empty_like(A)),
                         dict(spec=sb, A=A, B=W, C=torch.empty_like(B))]
        for mode in ("default", "split_bf16x3"):
            bt = comet.Batch(problems, dtype=f, compute=mode)
            bt()
            torch.cuda.synchronize()
            print("batch", mode, "done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="all", help="comma list of compute modes for the headline, or all")
    ap.add_argument("--only-headline", action="store_true", help="skip the other workloads")
    ap.add_argument("--sections", default="all",
                    help="comma list of the other workloads to run (backward, triples, config1, permute, "
                         "ttgt_study, chain, batch, batch_labels), all or none")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MB (HBM counter calibration)")
    ap.add_argument("--profile-pass", default="",
                    help="only run each named workload a few times, untimed, for a profiler's counter pass "
                         "(comma list of headline, split, triples, batch)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2102_06827_amd as comet

    if args.copy_mb:
        n = args.copy_mb * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}), flush=True)
        return

    if args.profile_pass:
        profile_pass(comet, args.profile_pass.split(","))
        return

    A, B, C0 = make_inputs()
    # bring the clocks up before anything is timed (about one second of work)
    Ah, Bh = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    t_end = time.perf_counter() + 1.0
    while time.perf_counter() < t_end:
        for _ in range(20):
            comet.contract(SPEC, Ah, Bh)
        torch.cuda.synchronize()
    del Ah, Bh
    torch.cuda.empty_cache()
    want = list(MODES) if args.modes == "all" else args.modes.split(",")
    if "f64" not in want:
        want = ["f64"] + want
    modes = bench_modes(comet, A, B, C0, args.steps, args.warmup, want)
    print("[bench] headline modes done", file=sys.stderr, flush=True)
    head = modes["f64"]
    ms = head["ms"]
    achieved = FLOPS / (ms * 1e-3) / 1e12
    Ad = torch.empty(shape("acik"), dtype=torch.float64, device="cuda")
    Bd = torch.empty(shape("bkcj"), dtype=torch.float64, device="cuda")
    sched = comet.Plan(SPEC, Ad, Bd, compute="f64").describe()
    sched = {k: sched[k] for k in ("path", "tile", "sk_tiles", "sk_blocks", "even", "even_whole", "resident")}
    del Ad, Bd
    same = (HEADLINE_TRAFFIC["kernel_version"] == KERNEL_VERSION and
            all(HEADLINE_TRAFFIC["schedule"][k] == sched[k] for k in HEADLINE_TRAFFIC["schedule"]))
    traffic = HEADLINE_TRAFFIC["bytes"] if same else None
    line = {
        "metric": "GFLOP/s & % MFMA peak per contraction: FP64 vs split-BF16x3 at stated rel err",
        "value": head["gflops"],
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
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["f64"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f64"], 4),
                     "traffic": traffic, "kernel": " + ".join(headline_kernels(sched)), "schedule": sched,
                     "algorithmic_flops": FLOPS, "algorithmic_bytes": 4 * 8.0 * V * V * O * O},
        "modes": modes,
    }
    if not args.only_headline:
        sections = {
            "backward": lambda: bench_backward(comet, A, B, C0, reps=5),
            "triples": lambda: bench_triples(comet, reps=5),
            "config1": lambda: bench_config1(comet),
            "permute": lambda: bench_permute(comet, reps=5),
            "ttgt_study": lambda: bench_ttgt_study(comet),
            "chain": lambda: bench_chain(comet),
            "batch": lambda: bench_batch(comet, reps=3),
            "batch_labels": lambda: bench_batch_labels(comet),
        }
        chosen = (list(sections) if args.sections == "all" else
                  [] if args.sections == "none" else args.sections.split(","))
        for name in chosen:
            if name not in sections:
                print("unknown section %r" % name, file=sys.stderr)
                sys.exit(2)
            t0 = time.perf_counter()
            line[name] = sections[name]()
            print("[bench] %s done in %.1f s" % (name, time.perf_counter() - t0), file=sys.stderr, flush=True)
    if not args.no_cpu:
        # the CPU leg: oracle references for every recorded check, and the
        # oracle's own throughput
        cpu_leg(line, A, B, C0)
        print("[bench] cpu leg done", file=sys.stderr, flush=True)
    if "config1" in line:
        line["config1"].pop("A")
        line["config1"].pop("B")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
