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
