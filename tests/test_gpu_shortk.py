"""The short-summation kernel (K <= 32; a persistent walk over 128 x 128
tiles whose stores overlap the next tile's products) against the oracle:
ragged M and N, every summation length up to 32, both storage types, both
operand layouts, beta 0 and beta != 0, fewer tiles than workgroups and
several per workgroup, a forced tile other than its own turning it off, and
the planner taking it for the triples contraction."""
import numpy as np
import pytest

from gpu_common import oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("spec,ext", [
    ("abcijk=daij*bcdk", dict(a=9, b=7, c=5, d=32, i=6, j=10, k=12)),   # the triples pattern, ragged
    ("abcijk=daij*bcdk", dict(a=4, b=3, c=2, d=17, i=16, j=8, k=16)),   # K = 17
    ("abcijk=daij*bcdk", dict(a=8, b=4, c=8, d=32, i=4, j=8, k=8)),     # whole tiles, K = 32: unmasked loads
    ("mn=km*kn", dict(m=300, n=520, k=4)),                              # both operands M/N-contiguous
    ("mn=mk*nk", dict(m=260, n=390, k=32)),                             # both K-contiguous
    ("mn=mk*kn", dict(m=1000, n=999, k=8)),
])
@pytest.mark.parametrize("beta", [0.0, -1.5])
def test_shortk_matches_oracle(spec, ext, dtype, beta, monkeypatch):
    c, a, b = oracle.split_spec(spec)
    A = synth.integers(7401, shape_of(a, ext))
    B = synth.integers(7402, shape_of(b, ext))
    C0 = synth.integers(7403, shape_of(c, ext))
    monkeypatch.setenv("COMET_GETT_SHORTK", "1")
    print_case("shortk", spec, dtype, beta)
    Ad, Bd, Cd = torch_dev(A, dtype), torch_dev(B, dtype), torch_dev(C0, dtype)
    plan = comet.Plan(spec, Ad, Bd, Cd, path="gett")
    d = plan.describe()
    if d["layoutA"] is not None and d["runs"]["Ak" if d["layoutA"] == "k" else "Am"] >= (2 if dtype == torch.float64 else 4) \
            and d["runs"]["Bk" if d["layoutB"] == "k" else "Bn"] >= (2 if dtype == torch.float64 else 4):
        assert d["shortk"] > 0 and d["tile"] == 3
    plan(Ad, Bd, Cd, alpha=2.0, beta=beta)
    torch.cuda.synchronize()
    ref = oracle.contract(spec, A, B, C0, alpha=2.0, beta=beta)
    assert np.array_equal(to_np(Cd), ref)


def test_shortk_chosen_for_triples_and_uniform_inputs():
    spec = "abcijk=daij*bcdk"
    ext = dict(a=32, b=32, c=32, d=32, i=16, j=16, k=16)
    c, a, b = oracle.split_spec(spec)
    A = synth.uniform(7411, shape_of(a, ext))
    B = synth.uniform(7412, shape_of(b, ext))
    print_case("shortk triples")
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    plan = comet.Plan(spec, Ad, Bd)
    assert plan.describe()["shortk"] > 0
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    shp = shape_of(c, ext)
    pts = np.stack([rng.integers(0, e, 2000) for e in shp], axis=1)
    pts = np.concatenate([pts, np.zeros((1, 6), np.int64), np.array([shp]) - 1])
    ref = oracle.contract_points(spec, A, B, pts)
    assert oracle.relerr(to_np(C)[tuple(pts.T)], ref) <= 1e-12


@pytest.mark.parametrize("spec,ext", [
    ("mn=km*kn", dict(m=4096, n=4096, k=32)),                           # 1024 whole tiles, row-contiguous operands
    ("abcijk=daij*bcdk", dict(a=16, b=16, c=16, d=32, i=16, j=16, k=16)),   # the triples pattern, 1024 whole tiles
    ("mn=km*kn", dict(m=4000, n=4100, k=32)),                           # ragged edges
])
def test_shortk_several_tiles_per_workgroup(spec, ext, monkeypatch):
    """Enough tiles that every workgroup walks several (beta = 0, whole tiles
    where the extents allow): integer inputs bit for bit."""
    c, a, b = oracle.split_spec(spec)
    A = synth.integers(7421, shape_of(a, ext))
    B = synth.integers(7422, shape_of(b, ext))
    monkeypatch.setenv("COMET_GETT_SHORTK", "1")
    print_case("shortk many tiles", spec)
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    plan = comet.Plan(spec, Ad, Bd, path="gett")
    d = plan.describe()
    assert d["shortk"] > 0 and d["tile"] == 3
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), oracle.contract(spec, A, B))


def test_forced_tile_turns_shortk_off(monkeypatch):
    """A forced tile other than the short-summation kernel's own (tile 3)
    keeps the plain schedule, which is still exact."""
    spec, ext = "mn=km*kn", dict(m=1024, n=1024, k=32)
    c, a, b = oracle.split_spec(spec)
    A = synth.integers(7431, shape_of(a, ext))
    B = synth.integers(7432, shape_of(b, ext))
    monkeypatch.setenv("COMET_GETT_SHORTK", "1")
    monkeypatch.setenv("COMET_GETT_TILE", "0")
    print_case("shortk forced tile 0")
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    plan = comet.Plan(spec, Ad, Bd, path="gett")
    d = plan.describe()
    assert d["shortk"] == 0 and d["tile"] == 0
    C = plan(Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), oracle.contract(spec, A, B))
