"""The autotuner: it times the tile variants and the TTGT lowering for a
problem class, records the winner in its JSON cache, reuses it, survives a
corrupt cache, and the tuned plan is still exact."""
import json

import numpy as np
import pytest

from gpu_common import oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")


@pytest.fixture
def cache(tmp_path):
    path = tmp_path / "tune.json"
    yield path
    comet.autotune(None, 0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_autotune_records_and_reuses(cache, dtype):
    spec = "abij=acik*bkcj"
    ext = dict(a=48, b=40, c=36, i=16, j=24, k=12)
    A = synth.integers(1, shape_of("acik", ext))
    B = synth.integers(2, shape_of("bkcj", ext))
    Ad, Bd = torch_dev(A, dtype), torch_dev(B, dtype)
    print_case("autotune", dtype)
    comet.autotune(str(cache), 1)
    plan = comet.Plan(spec, Ad, Bd)
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), oracle.contract(spec, A, B))
    data = json.loads(cache.read_text())
    assert data["format"] == "comet-tune-2" and len(data["entries"]) == 1
    (key, entry), = data["entries"].items()
    assert entry["path"] in (1, 2) and entry["us"] > 0
    chosen = plan.describe()
    assert chosen["path"] == ("ttgt" if entry["path"] == 2 else "gett")
    if entry["path"] == 1:
        assert chosen["tile"] == entry["tile"] and entry["ttgt"] == ""
    else:
        # the fastest of the timed flattenings, recorded and used
        t = chosen["ttgt"]
        assert entry["ttgt"] == "%s|%s|%s" % (t["A"], t["B"], t["C"])
    # a second plan of the same class reads the cache (no new entry, same choice)
    mtime = cache.stat().st_mtime_ns
    plan2 = comet.Plan(spec, Ad, Bd)
    assert plan2.describe()["path"] == chosen["path"]
    assert cache.stat().st_mtime_ns == mtime
    C2 = plan2(Ad, Bd)
    torch.cuda.synchronize()
    assert torch.equal(C, C2)


def test_autotune_rewrites_corrupt_cache(cache):
    cache.write_text('{"format": "comet-tune-2", "entries": {"x": {"tile": ')
    comet.autotune(str(cache), 1)
    A = torch_dev(synth.uniform(3, (200, 150)), torch.float64)
    B = torch_dev(synth.uniform(4, (150, 170)), torch.float64)
    print_case("autotune corrupt")
    C = comet.Plan("ij=ik*kj", A, B)(A, B)
    torch.cuda.synchronize()
    assert oracle.relerr(to_np(C), oracle.contract("ij=ik*kj", to_np(A), to_np(B))) <= 1e-12
    data = json.loads(cache.read_text())
    assert len(data["entries"]) == 1 and "x" not in data["entries"]


def test_autotune_searches_ttgt_flattenings(cache, monkeypatch):
    """With the gather path ruled out by forcing TTGT plans to compete only with
    each other (a problem whose TTGT flattenings differ), the recorded
    flattening is one of the candidates and the tuned plan is exact."""
    spec = "abcd=aebf*dfce"
    ext = dict(a=13, b=11, c=12, d=9, e=10, f=7)
    A = synth.integers(5, shape_of("aebf", ext))
    B = synth.integers(6, shape_of("dfce", ext))
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    print_case("autotune ttgt search")
    comet.autotune(str(cache), 2)
    plan = comet.Plan(spec, Ad, Bd)
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), oracle.contract(spec, A, B))
    (key, entry), = json.loads(cache.read_text())["entries"].items()
    if entry["path"] == 2:
        a, b, c = entry["ttgt"].split("|")
        assert sorted(a) == sorted("aebf") and sorted(b) == sorted("dfce") and sorted(c) == sorted("abcd")


@pytest.mark.parametrize("dtype,choices", [(torch.float64, (0, 1)), (torch.float32, (0, 1, 2))])
def test_autotune_split_product_tile(cache, dtype, choices):
    """The classic BF16x3 split: the slice-pair tiles (and, on FP32 storage,
    the fused kernel) are timed, the winner is recorded and used, and the
    tuned plan is exact on integer inputs."""
    spec = "abij=acik*bkcj"
    ext = dict(a=40, b=36, c=24, i=12, j=16, k=20)
    A = synth.integers(11, shape_of("acik", ext))
    B = synth.integers(12, shape_of("bkcj", ext))
    Ad, Bd = torch_dev(A, dtype), torch_dev(B, dtype)
    print_case("autotune split", dtype)
    comet.autotune(str(cache), 2)
    plan = comet.Plan(spec, Ad, Bd, compute="split_bf16x3")
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), oracle.contract(spec, A, B))
    (key, entry), = json.loads(cache.read_text())["entries"].items()
    assert entry["tile"] in choices and entry["us"] > 0 and "/c4/" in key
    d = plan.describe()
    assert d["fused3"] == (entry["tile"] == 2)
    if entry["tile"] != 2:
        assert d["split_tile"] == entry["tile"]


def test_autotune_aligned_split_tile(cache):
    """The aligned BF16 split: the 128 x 64 and 128 x 96 slice-pair tiles are
    timed, the winner is recorded and used, and the tuned plan is exact on
    integer inputs."""
    spec = "abij=acik*bkcj"
    ext = dict(a=40, b=36, c=24, i=12, j=16, k=20)
    A = synth.integers(13, shape_of("acik", ext))
    B = synth.integers(14, shape_of("bkcj", ext))
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    print_case("autotune aligned split")
    comet.autotune(str(cache), 2)
    plan = comet.Plan(spec, Ad, Bd, compute="split_bf16")
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), oracle.contract(spec, A, B))
    (key, entry), = json.loads(cache.read_text())["entries"].items()
    assert entry["tile"] in (0, 2) and entry["us"] > 0
    assert plan.describe()["split_tile"] == entry["tile"]


def test_autotune_ttgt_flattening(cache):
    """A plan that asks for TTGT with the autotuner on: every flattening is
    timed, the fastest is recorded under its own key and used (also from the
    cache), and the result is exact on integer inputs."""
    spec = "abij=acik*bkcj"
    ext = dict(a=16, b=12, c=8, i=8, j=12, k=8)
    A = synth.integers(15, shape_of("acik", ext))
    B = synth.integers(16, shape_of("bkcj", ext))
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    ref = oracle.contract(spec, A, B)
    print_case("autotune ttgt flattening")
    comet.autotune(str(cache), 2)
    plan = comet.Plan(spec, Ad, Bd, path="ttgt")
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), ref)
    (key, entry), = json.loads(cache.read_text())["entries"].items()
    assert key.endswith("/ttgt") and entry["path"] == 2 and entry["us"] > 0
    t = plan.describe()["ttgt"]
    assert entry["ttgt"] == "%s|%s|%s" % (t["A"], t["B"], t["C"])
    # from the cache: the same flattening, no new entry
    comet.autotune(str(cache), 1)
    plan2 = comet.Plan(spec, Ad, Bd, path="ttgt")
    t2 = plan2.describe()["ttgt"]
    assert (t2["A"], t2["B"], t2["C"]) == (t["A"], t["B"], t["C"])
    assert np.array_equal(to_np(plan2(Ad, Bd)), ref)
    assert len(json.loads(cache.read_text())["entries"]) == 1


def test_autotune_batch_classes(cache):
    """The batch's tile classes come from timings per problem class: every
    problem is counted as tuned, the cache holds batch entries with valid
    classes, a second batch reuses them without timing, and results are
    exact on integer inputs."""
    rng = np.random.default_rng(2)
    host, dev = [], []
    for t in range(10):
        spec = ["abij=acik*bkcj", "abij=abcd*cdij"][t % 2]
        c, a, b = oracle.split_spec(spec)
        ext = {ch: int(rng.choice([8, 24, 64])) for ch in set(a + b)}
        A = synth.integers(20 + t, shape_of(a, ext)).astype(np.float32)
        B = synth.integers(40 + t, shape_of(b, ext)).astype(np.float32)
        host.append((spec, A, B))
        C = torch.zeros(shape_of(c, ext), dtype=torch.float32, device="cuda")
        dev.append(dict(spec=spec, A=torch_dev(A, torch.float32), B=torch_dev(B, torch.float32), C=C))
    print_case("autotune batch")
    comet.autotune(str(cache), 1)
    bt = comet.Batch(dev, dtype=torch.float32)
    d = bt.describe()
    assert d["tuned"] == len(dev)
    entries = json.loads(cache.read_text())["entries"]
    batch_entries = {k: v for k, v in entries.items() if k.startswith("batch/")}
    assert batch_entries and all(0 <= v["tile"] <= 3 and v["us"] > 0 for v in batch_entries.values())
    mtime = cache.stat().st_mtime_ns
    bt2 = comet.Batch(dev, dtype=torch.float32)
    assert bt2.describe()["classes"] == d["classes"] and cache.stat().st_mtime_ns == mtime
    bt()
    torch.cuda.synchronize()
    for (spec, A, B), x in zip(host, dev):
        assert np.array_equal(to_np(x["C"]), oracle.contract(spec, A, B)), spec


def test_autotune_environment_switch(tmp_path):
    """COMET_AUTOTUNE=on turns the autotuner on from the environment (a fresh
    process), with the cache at COMET_TUNE_CACHE."""
    import os
    import subprocess
    import sys
    path = tmp_path / "env_tune.json"
    code = ("import torch, paper_2102_06827_amd as c; "
            "A = torch.ones(64, 96, dtype=torch.float64, device='cuda'); "
            "B = torch.ones(96, 80, dtype=torch.float64, device='cuda'); "
            "C = c.contract('ij=ik*kj', A, B); torch.cuda.synchronize(); "
            "assert bool((C == 96).all())")
    env = dict(os.environ, COMET_AUTOTUNE="on", COMET_TUNE_CACHE=str(path))
    print_case("autotune env")
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=os.path.dirname(os.path.dirname(__file__)),
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert len(json.loads(path.read_text())["entries"]) == 1
