"""The planner's automatic TTGT lowering for contractions that only the
element-load gather kernel can read, at either side of its cost estimate,
and the convenience call's per-stream workspaces."""
import numpy as np
import pytest

from gpu_common import oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

# A[c,d,m,n] is contiguous along n, B[i,n,a,d] along d: both unit strides are
# summation labels, but different ones, so no summation order gives both
# operands vector reads -- the gather path needs its element-load kernel
SPEC = "cmia=cdmn*inad"


def _ext(cm, ia, dn):
    (c, m), (i, a), (d, n) = cm, ia, dn
    return dict(c=c, m=m, i=i, a=a, d=d, n=n)


@pytest.mark.parametrize("dtype,sizes,path", [
    (torch.float64, ((16, 32), (16, 32), (16, 32)), "gett"),    # 512^3: permutes cost more than they save
    (torch.float64, ((24, 32), (24, 32), (24, 32)), "ttgt"),    # 768^3
    (torch.float32, ((16, 32), (16, 32), (16, 32)), "gett"),
    (torch.float32, ((24, 32), (24, 32), (24, 32)), "ttgt"),
    # 4096^2 x 16, C in the product's own order: TTGT only permutes the two
    # small operands
    (torch.float64, ((64, 64), (64, 64), (4, 4)), "ttgt"),
    # odd extents: not even the TTGT matrices can be read in vectors, but
    # their GEMM still reads dense rows (3025^3: 1.2 against 4.2 ms gathered)
    (torch.float64, ((45, 45), (45, 45), (45, 45)), "ttgt"),
    (torch.float32, ((45, 45), (45, 45), (45, 45)), "ttgt"),
])
def test_auto_ttgt_switch_follows_the_estimate(dtype, sizes, path):
    _check_switch(SPEC, dtype, sizes, path)


def test_auto_ttgt_switch_keeps_gather_when_C_would_move():
    # the same short summation with C's free labels interleaved (c, i, m, a):
    # TTGT would have to permute the 134 MB output, so the gather path stays
    _check_switch("cima=cdmn*inad", torch.float64, ((64, 64), (64, 64), (4, 4)), "gett")


def _check_switch(spec, dtype, sizes, path):
    ext = _ext(*sizes)
    SPEC_ = spec
    c, a, b = oracle.split_spec(SPEC_)
    A = synth.integers(8101, shape_of(a, ext))
    B = synth.integers(8102, shape_of(b, ext))
    print_case("ttgt switch", dtype, sizes)
    Ad, Bd = torch_dev(A, dtype), torch_dev(B, dtype)
    plan = comet.Plan(SPEC_, Ad, Bd)
    assert plan.describe()["path"] == path
    got = plan(Ad, Bd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    shp = shape_of(c, ext)
    pts = np.stack([rng.integers(0, e, 512) for e in shp], axis=1)
    pts = np.concatenate([pts, np.zeros((1, len(shp)), np.int64), np.array([shp]) - 1])
    ref = oracle.contract_points(SPEC_, A, B, pts)
    g = to_np(got)
    assert np.array_equal(g[tuple(pts.T)], ref)


def test_forced_gather_tile_keeps_the_gather_path(monkeypatch):
    ext = _ext((24, 32), (24, 32), (24, 32))
    c, a, b = oracle.split_spec(SPEC)
    A = synth.integers(8111, shape_of(a, ext))
    B = synth.integers(8112, shape_of(b, ext))
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    monkeypatch.setenv("COMET_GETT_TILE", "1")
    print_case("ttgt switch forced tile")
    plan = comet.Plan(SPEC, Ad, Bd)
    d = plan.describe()
    assert d["path"] == "gett" and d["tile"] == 1
    # the element-load variant keeps whole tiles when forced (its stream-K
    # split is for latency-bound problems only)
    assert d["sk_tiles"] == 0
    got = plan(Ad, Bd)
    torch.cuda.synchronize()
    pts = np.array([[0] * 4, [x - 1 for x in shape_of(c, ext)], [3, 5, 7, 11]])
    assert np.array_equal(to_np(got)[tuple(pts.T)], oracle.contract_points(SPEC, A, B, pts))


def test_convenience_call_on_two_streams_does_not_share_workspace():
    """Two streams alternately run contractions whose plans need workspace
    (aligned BF16 slices), with no ordering between the streams: each
    result matches its own oracle."""
    spec = "abij=acik*bkcj"
    cases = []
    for t, (V, O) in enumerate(((40, 12), (36, 16))):
        ext = dict(a=V, b=V, c=V, i=O, j=O, k=O)
        A = synth.uniform(8200 + 10 * t, shape_of("acik", ext))
        B = synth.uniform(8201 + 10 * t, shape_of("bkcj", ext))
        cases.append((A, B, oracle.contract(spec, A, B)))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    print_case("two streams")
    dev = [(torch_dev(A, torch.float64), torch_dev(B, torch.float64)) for A, B, _ in cases]
    torch.cuda.synchronize()
    outs = [[], []]
    for rep in range(6):
        for t in (0, 1):
            with torch.cuda.stream(streams[t]):
                outs[t].append(comet.contract(spec, dev[t][0], dev[t][1], compute="split_bf16",
                                              stream=streams[t]))
    torch.cuda.synchronize()
    for t in (0, 1):
        for C in outs[t]:
            assert oracle.relerr(to_np(C), cases[t][2]) <= 1e-9
