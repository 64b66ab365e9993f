"""Parity of the HIP contraction path against the CPU FP64 oracle.

Bars: relative Frobenius error <= 1e-12 for FP64 arithmetic and <= 1e-5 for
FP32 arithmetic; bit-exact results for integer-valued inputs (every partial
sum is an exact integer in both precisions) and for the pure data-movement
permute kernel.
"""
import os
import random

import numpy as np
import pytest

from gpu_common import TOL, inputs, oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

DT = {"f64": None, "f32": None}


def tdt(name):
    return torch.float64 if name == "f64" else torch.float32


def run(spec, A, B, C0=None, alpha=1.0, beta=0.0, dtype="f64", compute="default", path=None):
    Ad, Bd = torch_dev(A, tdt(dtype)), torch_dev(B, tdt(dtype))
    Cd = torch_dev(C0, tdt(dtype)) if C0 is not None else None
    if path is None:
        out = comet.contract(spec, Ad, Bd, Cd, alpha=alpha, beta=beta, compute=compute)
    else:
        plan = comet.Plan(spec, Ad, Bd, Cd, compute=compute, path=path)
        out = plan(Ad, Bd, Cd, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    return to_np(out)


def ref_of(spec, A, B, C0, alpha, beta, dtype):
    """Oracle on exactly the values the GPU received (rounded to storage)."""
    cast = np.float32 if dtype == "f32" else np.float64
    Ar, Br = A.astype(cast), B.astype(cast)
    Cr = C0.astype(cast) if C0 is not None else None
    return oracle.contract(spec, Ar, Br, Cr, alpha=alpha, beta=beta)


def check(spec, ext, dtype, seed, kind="uniform", alpha=1.0, beta=0.0, compute="default", path=None):
    print_case(spec, ext, dtype, kind, "alpha", alpha, "beta", beta, compute, path)
    A, B, C0 = inputs(spec, ext, seed, kind=kind, beta=True)
    got = run(spec, A, B, C0, alpha, beta, dtype, compute, path)
    ref = ref_of(spec, A, B, C0, alpha, beta, dtype)
    assert got.shape == ref.shape
    if kind == "integer":
        assert np.array_equal(got, ref), "integer inputs must match bit for bit"
    else:
        mode = dtype if compute == "default" else compute
        err = oracle.relerr(got, ref)
        assert err <= TOL[mode], "relerr %.3e > %.0e" % (err, TOL[mode])
    return got


CONFIG_SMALL = [
    # config 1 at full size (all extents 16)
    ("abij=acik*cbkj", dict(a=16, b=16, c=16, i=16, j=16, k=16)),
    # config 2 shape family, several tiles plus a ragged tail (M = N = K = 480)
    ("abij=acik*bkcj", dict(a=40, b=40, c=40, i=12, j=12, k=12)),
    # config 3 shape family, ragged
    ("abcijk=daij*bcdk", dict(a=10, b=9, c=7, d=12, i=6, j=5, k=6)),
    # config 5 patterns
    ("abij=abcd*cdij", dict(a=9, b=13, c=7, d=11, i=10, j=14)),
    ("abij=ijcd*cdab", dict(a=9, b=13, c=7, d=11, i=10, j=14)),
    ("abij=ciak*bkjc", dict(a=17, b=9, c=12, i=8, j=24, k=6)),
    ("ajbi=kcia*cjkb", dict(a=17, b=9, c=12, i=8, j=24, k=6)),
    # the paper's worked example
    ("abcd=aebf*dfce", dict(a=13, b=11, c=12, d=9, e=10, f=7)),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", CONFIG_SMALL)
def test_configs_random(spec, ext, dtype):
    check(spec, ext, dtype, seed=100, beta=1.0, alpha=0.75)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", CONFIG_SMALL)
def test_configs_integer_bitwise(spec, ext, dtype):
    check(spec, ext, dtype, seed=200, kind="integer", beta=1.0, alpha=1.0)


@pytest.mark.parametrize("compute", ["f64", "f32"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cross_precision(dtype, compute):
    spec, ext = CONFIG_SMALL[1]
    A, B, C0 = inputs(spec, ext, 300, beta=True)
    print_case("cross", dtype, compute)
    got = run(spec, A, B, C0, 1.0, 1.0, dtype, compute)
    ref = ref_of(spec, A, B, C0, 1.0, 1.0, dtype)
    tol = 1e-5 if (compute == "f32" or dtype == "f32") else 1e-12
    assert oracle.relerr(got, ref) <= tol


def random_spec(rng, max_per_class=3):
    letters = list("abcdefghijklmnopqrstuvwxyz")
    rng.shuffle(letters)
    nm, nn, nk = rng.randint(0, max_per_class), rng.randint(0, max_per_class), rng.randint(0, max_per_class)
    m, n, k = letters[:nm], letters[nm:nm + nn], letters[nm + nn:nm + nn + nk]
    a, b, c = m + k, k + n, m + n
    rng.shuffle(a)
    rng.shuffle(b)
    rng.shuffle(c)
    return "%s=%s*%s" % ("".join(c), "".join(a), "".join(b))


@pytest.mark.parametrize("case", range(40))
def test_random_specs(case):
    rng = random.Random(5000 + case)
    spec = random_spec(rng)
    ext = {ch: rng.randint(1, 9) for ch in set(spec) if ch.isalpha()}
    dtype = "f64" if case % 2 == 0 else "f32"
    kind = "integer" if case % 3 == 0 else "uniform"
    check(spec, ext, dtype, seed=6000 + case, kind=kind, alpha=rng.choice([1.0, -0.5, 2.0]),
          beta=rng.choice([0.0, 1.0, -1.5]))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_strided_views(dtype):
    spec = "abij=acik*bkcj"
    ext = dict(a=20, b=18, c=22, i=9, j=7, k=10)
    base_A = synth.uniform(11, (26, 30, 12, 14))
    base_B = synth.uniform(12, (20, 12, 25, 9))
    base_C = synth.uniform(13, (22, 21, 11, 9))
    Ad = torch_dev(base_A, tdt(dtype))[1:21, 2:24, 1:10, 3:13]
    Bd = torch_dev(base_B, tdt(dtype))[0:18, 1:11, 2:24, 1:8]
    Cfull = torch_dev(base_C, tdt(dtype))
    Cd = Cfull[1:21, 2:20, 1:10, 1:8]
    print_case("strided", dtype)
    A, B, C0 = to_np(Ad), to_np(Bd), to_np(Cd)
    comet.contract(spec, Ad, Bd, Cd, alpha=1.0, beta=1.0)
    torch.cuda.synchronize()
    ref = oracle.contract(spec, A, B, C0, alpha=1.0, beta=1.0)
    assert oracle.relerr(to_np(Cd), ref) <= TOL[dtype]
    # the rest of the big C buffer is untouched
    Cf = to_np(Cfull)
    mask = np.ones(Cf.shape, bool)
    mask[1:21, 2:20, 1:10, 1:8] = False
    assert np.array_equal(Cf[mask], base_C.astype(np.float32 if dtype == "f32" else np.float64)[mask])


def test_beta_zero_ignores_nan_in_C():
    spec, ext = CONFIG_SMALL[0]
    A, B, _ = inputs(spec, ext, 21)
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    Cd = torch.full(shape_of("abij", ext), float("nan"), dtype=torch.float64, device="cuda")
    print_case("beta0 nan")
    comet.contract(spec, Ad, Bd, Cd, beta=0.0)
    torch.cuda.synchronize()
    assert torch.isfinite(Cd).all()
    assert oracle.relerr(to_np(Cd), oracle.contract(spec, A, B)) <= 1e-12


def test_alpha_zero_scales_C_only():
    spec, ext = CONFIG_SMALL[0]
    C0 = synth.uniform(22, shape_of("abij", ext))
    Ad = torch.full(shape_of("acik", ext), float("nan"), dtype=torch.float64, device="cuda")
    Bd = torch.full(shape_of("cbkj", ext), float("nan"), dtype=torch.float64, device="cuda")
    Cd = torch_dev(C0, torch.float64)
    print_case("alpha0")
    comet.contract(spec, Ad, Bd, Cd, alpha=0.0, beta=2.0)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(Cd), 2.0 * C0)


def test_empty_and_degenerate():
    print_case("degenerate")
    # zero contracted extent: C = beta * C
    A = torch.zeros((5, 0), dtype=torch.float64, device="cuda")
    B = torch.zeros((0, 7), dtype=torch.float64, device="cuda")
    C0 = synth.uniform(31, (5, 7))
    C = torch_dev(C0, torch.float64)
    comet.contract("ij=ik*kj", A, B, C, beta=3.0)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), 3.0 * C0)
    # zero free extent: nothing happens, no error
    A = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    B = torch.ones((4, 3), dtype=torch.float64, device="cuda")
    C = comet.contract("ij=ik*kj", A, B)
    assert C.shape == (0, 3)
    # full contraction to a scalar
    Ai = synth.integers(32, (37, 41))
    Bi = synth.integers(33, (41, 37))
    C = comet.contract("=ab*ba", torch_dev(Ai, torch.float64), torch_dev(Bi, torch.float64))
    torch.cuda.synchronize()
    assert float(C.item()) == float(np.sum(Ai * Bi.T))
    # outer product
    A = synth.uniform(34, (13, 6))
    B = synth.uniform(35, (9,))
    C = comet.contract("iaj=ij*a", torch_dev(A, torch.float64), torch_dev(B, torch.float64))
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), A[:, None, :] * B[None, :, None])
    # extent-1 labels everywhere
    check("abij=acik*cbkj", dict(a=1, b=1, c=1, i=1, j=1, k=1), "f64", 36)
    check("abij=acik*cbkj", dict(a=1, b=7, c=1, i=5, j=1, k=3), "f64", 37)


@pytest.mark.parametrize("spec,ext", [CONFIG_SMALL[1], CONFIG_SMALL[2], CONFIG_SMALL[7], CONFIG_SMALL[6]])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ttgt_equals_gett_and_oracle(spec, ext, dtype):
    A, B, C0 = inputs(spec, ext, 400, beta=True)
    print_case("ttgt", spec, dtype)
    g = run(spec, A, B, C0, 1.25, -1.0, dtype, path="gett")
    t = run(spec, A, B, C0, 1.25, -1.0, dtype, path="ttgt")
    ref = ref_of(spec, A, B, C0, 1.25, -1.0, dtype)
    assert oracle.relerr(g, ref) <= TOL[dtype]
    assert oracle.relerr(t, ref) <= TOL[dtype]
    Ai, Bi, Ci = inputs(spec, ext, 401, kind="integer", beta=True)
    gi = run(spec, Ai, Bi, Ci, 1.0, 1.0, dtype, path="gett")
    ti = run(spec, Ai, Bi, Ci, 1.0, 1.0, dtype, path="ttgt")
    assert np.array_equal(gi, ti)
    assert np.array_equal(gi, ref_of(spec, Ai, Bi, Ci, 1.0, 1.0, dtype))


def test_ttgt_with_the_papers_worked_example_permutation(monkeypatch):
    """TTGT forced to the decomposition printed for the worked example
    (TA[a,b,e,f], TB[e,f,d,c], TC[a,b,d,c]) equals the oracle."""
    spec = "abcd=aebf*dfce"
    ext = dict(a=13, b=11, c=12, d=9, e=10, f=7)
    monkeypatch.setenv("COMET_TTGT_ORDER", "abef|efdc|abdc")
    A, B, C0 = inputs(spec, ext, 410, kind="integer", beta=True)
    print_case("ttgt paper order")
    got = run(spec, A, B, C0, 1.0, 1.0, "f64", path="ttgt")
    assert np.array_equal(got, ref_of(spec, A, B, C0, 1.0, 1.0, "f64"))


def test_determinism_bitwise():
    spec, ext = CONFIG_SMALL[1]
    A, B, C0 = inputs(spec, ext, 500, beta=True)
    print_case("determinism")
    r1 = run(spec, A, B, C0, 1.0, 1.0, "f64")
    r2 = run(spec, A, B, C0, 1.0, 1.0, "f64")
    assert np.array_equal(r1, r2)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,shape", [
    ("ji=ij", (67, 45)),
    ("kji=ijk", (33, 17, 29)),
    ("acbd=abcd", (5, 34, 40, 3)),
    ("dcba=abcd", (7, 9, 11, 35)),
    ("bcda=abcd", (40, 3, 5, 7)),
    ("abcd=abcd", (3, 4, 5, 6)),
    # shared unit dimension, short rows (vector and element streams)
    ("aick=acik", (5, 6, 7, 8)),
    ("abcijk=aijbck", (3, 2, 5, 4, 3, 16)),
    ("bac=abc", (9, 7, 5)),
    # unit dimensions shorter than the tile: merged input / output groups
    ("abij=ijab", (5, 6, 7, 8)),
    ("fedcba=abcdef", (3, 4, 2, 5, 3, 6)),
    ("cadb=abcd", (2, 3, 33, 4)),
])
def test_permute_bitwise(spec, shape, dtype):
    lo, li = spec.split("=")
    x = synth.uniform(600, shape)
    xd = torch_dev(x, tdt(dtype))
    print_case("permute", spec, dtype)
    out = comet.permute(spec, xd)
    torch.cuda.synchronize()
    ref = np.transpose(x.astype(np.float32 if dtype == "f32" else np.float64), [li.index(ch) for ch in lo])
    assert np.array_equal(to_np(out), ref)
    # alpha, beta
    o0 = synth.uniform(601, ref.shape)
    od = torch_dev(o0, tdt(dtype))
    comet.permute(spec, xd, od, alpha=2.0, beta=-1.0)
    torch.cuda.synchronize()
    cast = np.float32 if dtype == "f32" else np.float64
    exp = (2.0 * ref.astype(np.float64) - o0.astype(cast).astype(np.float64)).astype(cast)
    assert np.array_equal(to_np(od).astype(cast), exp)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_permute_views_broadcast_and_scaling(dtype):
    """Strided views on both sides, a broadcast (stride 0) input, alpha = 0."""
    t = tdt(dtype)
    big = torch_dev(synth.uniform(610, (12, 30, 20)), t)
    x = big[1:11, ::3, 2:18]                       # (10, 10, 16), non-dense strides
    obig = torch.zeros((20, 12, 40), dtype=t, device="cuda")
    out = obig[2:18, 1:11, ::4]                    # (16, 10, 10) view
    print_case("permute views", dtype)
    comet.permute("cab=abc", x, out)
    torch.cuda.synchronize()
    assert torch.equal(out, x.permute(2, 0, 1))
    assert torch.count_nonzero(obig).item() == torch.count_nonzero(out).item()   # nothing outside the view
    col = torch_dev(synth.uniform(611, (7, 1)), t).expand(7, 9)   # stride (1, 0)
    r = comet.permute("ji=ij", col)
    torch.cuda.synchronize()
    assert torch.equal(r, col.t())
    o = torch_dev(synth.uniform(612, (9, 7)), t)
    ref = o * 0.5
    comet.permute("ji=ij", col, o, alpha=0.0, beta=0.5)
    torch.cuda.synchronize()
    assert torch.equal(o, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fill(dtype):
    """comet_fill: dense, a strided view (nothing outside it changes), rank 0,
    the FP32 rounding of the value."""
    t = tdt(dtype)
    x = torch.zeros((7, 9, 5), dtype=t, device="cuda")
    print_case("fill", dtype)
    comet.fill(x, -2.5)
    torch.cuda.synchronize()
    assert torch.equal(x, torch.full_like(x, -2.5))
    big = torch.zeros((12, 30), dtype=t, device="cuda")
    v = big[2:9, 1::3]
    comet.fill(v, 1.0 / 3.0)
    torch.cuda.synchronize()
    exp = torch.zeros_like(big)
    exp[2:9, 1::3] = torch.tensor(1.0 / 3.0, dtype=t)
    assert torch.equal(big, exp)
    s = torch.zeros((), dtype=t, device="cuda")
    comet.fill(s, 7.0)
    torch.cuda.synchronize()
    assert s.item() == 7.0
    odd = torch.zeros((3, 5, 7), dtype=t, device="cuda").permute(2, 0, 1)
    comet.fill(odd, 4.0)
    torch.cuda.synchronize()
    assert torch.equal(odd, torch.full_like(odd, 4.0))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_contiguous_fill_and_copy(dtype):
    """One contiguous run on both sides (the plain vector walk): a fill of
    40M elements (several grid passes), a scaled copy with beta != 0, and the
    same run one element off 16-byte alignment (the table-driven kernel)."""
    t = tdt(dtype)
    x = torch.zeros(40_000_004, dtype=t, device="cuda")
    print_case("contiguous fill", dtype)
    comet.fill(x, 3.25)
    torch.cuda.synchronize()
    assert torch.equal(x, torch.full_like(x, 3.25))
    del x
    a = synth.uniform(620, (1000, 1004))
    o0 = synth.uniform(621, (1000, 1004))
    ad, od = torch_dev(a, t), torch_dev(o0, t)
    comet.permute("ab=ab", ad, od, alpha=2.0, beta=-1.0)
    torch.cuda.synchronize()
    cast = np.float32 if dtype == "f32" else np.float64
    exp = (2.0 * a.astype(cast).astype(np.float64) - o0.astype(cast).astype(np.float64)).astype(cast)
    assert np.array_equal(to_np(od).astype(cast), exp)
    buf = torch.zeros(1002, dtype=t, device="cuda")
    v = buf[1:1001]
    comet.fill(v, -1.5)
    torch.cuda.synchronize()
    assert buf[0].item() == 0.0 and buf[1001].item() == 0.0 and torch.equal(v, torch.full_like(v, -1.5))


@pytest.mark.parametrize("spec", ["ji=ij", "jik=ijk"])
def test_permute_64bit_indexing(spec):
    """More than 2^30 elements: the 64-bit index path of both kernels."""
    if spec == "ji=ij":
        x = torch.empty((32768, 32776), dtype=torch.float32, device="cuda")
    else:
        x = torch.empty((1024, 1024, 1040), dtype=torch.float32, device="cuda")
    assert x.numel() > (1 << 30)
    x.copy_(torch.arange(x.numel(), device="cuda", dtype=torch.float32).view(x.shape) % 8191)
    print_case("permute 64-bit", spec)
    out = comet.permute(spec, x)
    torch.cuda.synchronize()
    lo, li = spec.split("=")
    assert torch.equal(out, x.permute(*[li.index(c) for c in lo]))
    del x, out
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# full-size configurations, sampled against the oracle
# --------------------------------------------------------------------------

def sample_points(shape, n, seed):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, s, n) for s in shape], axis=1)
    # always include the corners of the index space
    pts[0] = 0
    pts[1] = np.array(shape) - 1
    return pts


def config2_inputs():
    V, O = 96, 32
    ext = dict(a=V, b=V, c=V, i=O, j=O, k=O)
    A = synth.decayed_normal(synth.config_seed(2, "A"), "acik", shape_of("acik", ext), "abc", "ijk")
    B = synth.decayed_normal(synth.config_seed(2, "B"), "bkcj", shape_of("bkcj", ext), "abc", "ijk")
    C0 = synth.decayed_normal(synth.config_seed(2, "C0"), "abij", shape_of("abij", ext), "abc", "ijk")
    return ext, A, B, C0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_config2_full_size_sampled(dtype):
    spec = "abij=acik*bkcj"
    ext, A, B, C0 = config2_inputs()
    print_case("config2 full", dtype)
    got = run(spec, A, B, C0, 1.0, 1.0, dtype)
    cast = np.float32 if dtype == "f32" else np.float64
    pts = sample_points(got.shape, 3000, 7)
    ref = oracle.contract_points(spec, A.astype(cast), B.astype(cast), pts, C0.astype(cast), 1.0, 1.0)
    g = got[tuple(pts.T)]
    assert oracle.relerr(g, ref) <= TOL[dtype]
    # the beta = 0 product alone, so C0 cannot hide product errors
    got0 = run(spec, A, B, None, 1.0, 0.0, dtype)
    ref0 = oracle.contract_points(spec, A.astype(cast), B.astype(cast), pts)
    assert oracle.relerr(got0[tuple(pts.T)], ref0) <= TOL[dtype]


def test_config3_full_size_sampled():
    spec = "abcijk=daij*bcdk"
    ext = dict(a=32, b=32, c=32, d=32, i=16, j=16, k=16)
    A = synth.uniform(synth.config_seed(3, "A"), shape_of("daij", ext))
    B = synth.uniform(synth.config_seed(3, "B"), shape_of("bcdk", ext))
    print_case("config3 full")
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    C = comet.contract(spec, Ad, Bd)
    torch.cuda.synchronize()
    pts = sample_points(tuple(C.shape), 4000, 8)
    idx = torch.from_numpy(pts).cuda()
    g = C[tuple(idx.T)].cpu().numpy()
    ref = oracle.contract_points(spec, A, B, pts)
    assert oracle.relerr(g, ref) <= 1e-12
    # all-ones closed form over the whole output: every element is d = 32
    C1 = comet.contract(spec, torch.ones_like(Ad), torch.ones_like(Bd))
    torch.cuda.synchronize()
    assert bool((C1 == 32.0).all())
    del C, C1


def test_config1_oracle_and_delta():
    spec = "abij=acik*cbkj"
    n = 16
    A = synth.uniform(1001, (n,) * 4)
    B = np.einsum("cb,kj->cbkj", np.eye(n), np.eye(n))
    print_case("config1 delta")
    got = run(spec, A, B)
    assert np.array_equal(got, A)


@pytest.mark.parametrize("tile", range(10))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", [
    ("abij=acik*bkcj", dict(a=21, b=19, c=23, i=13, j=11, k=9)),      # A k-contiguous, B n-contiguous
    ("ajbi=kcia*cjkb", dict(a=18, b=9, c=12, i=16, j=24, k=6)),       # A m-contiguous (after the swap)
    ("abij=ijcd*cdab", dict(a=9, b=13, c=7, d=11, i=10, j=14)),       # B k-contiguous
])
def test_tile_variants(tile, dtype, spec, ext, monkeypatch):
    """Every GETT tile variant, on all operand layouts, with ragged edges."""
    monkeypatch.setenv("COMET_GETT_TILE", str(tile))
    check(spec, ext, dtype, seed=700 + tile, kind="integer", alpha=1.0, beta=1.0)
    check(spec, ext, dtype, seed=720 + tile, alpha=-0.5, beta=0.25)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", [
    ("abij=acik*bkcj", dict(a=16, b=24, c=8, i=16, j=16, k=6)),      # A k-contiguous, B n-contiguous
    ("ajbi=kcia*cjkb", dict(a=16, b=16, c=4, i=16, j=24, k=8)),       # A m-contiguous (after the swap)
    ("abij=ijcd*cdab", dict(a=16, b=8, c=4, d=12, i=8, j=32)),        # B k-contiguous
    ("abij=acik*cbkj", dict(a=16, b=16, c=8, i=8, j=8, k=4)),         # both m/n-contiguous
])
@pytest.mark.parametrize("tile", [3, 4])
def test_whole_tiles_unmasked_loads(tile, dtype, spec, ext, monkeypatch):
    """Outputs that are whole tiles with a summation of whole 16-index
    steps: tile 3 (128 x 128) takes the unmasked loads for its whole tiles,
    tile 4 (256 x 128) the masked ones on the same shapes; whole and in a
    forced stream-K split (which keeps masked loads): bit-exact on integer
    inputs, within the bar on uniform ones."""
    monkeypatch.setenv("COMET_GETT_TILE", str(tile))
    check(spec, ext, dtype, seed=1100, kind="integer", alpha=1.0, beta=1.0)
    check(spec, ext, dtype, seed=1110, alpha=-0.5, beta=0.25)
    monkeypatch.setenv("COMET_GETT_SK", "2,5")
    check(spec, ext, dtype, seed=1140, kind="integer", alpha=1.5, beta=-1.0, path="gett")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_whole_tiles_unmasked_loads_in_pieces(dtype, monkeypatch):
    """Six whole tiles over a long summation (K = 5504 = 344 steps), cut into
    the balanced schedule's pieces: the pieces' unmasked loads run over k
    tables moved to each piece's first index."""
    monkeypatch.setenv("COMET_GETT_TILE", "3")
    monkeypatch.setenv("COMET_GETT_EVEN", "1")
    spec, ext = "abij=acik*bkcj", dict(a=16, b=24, c=86, i=16, j=16, k=64)
    A = torch.zeros(shape_of("acik", ext), dtype=torch.float64, device="cuda")
    B = torch.zeros(shape_of("bkcj", ext), dtype=torch.float64, device="cuda")
    d = comet.Plan(spec, A, B, path="gett").describe()
    if dtype == "f64":
        assert d["even"] == 1 and d["sk_tiles"] == 6, d
    check(spec, ext, dtype, seed=1120, kind="integer", alpha=2.0, beta=1.0, path="gett")
    check(spec, ext, dtype, seed=1130, alpha=0.5, beta=0.0, path="gett")


SK_CASES = [
    # (tile, "tiles,blocks") on a 480 x 480 x 480 contraction with ragged edges:
    # shares inside one tile, shares over tile boundaries, more blocks than
    # steps (empty shares), a single block, every tile split
    (3, "4,16"), (3, "9,5"), (3, "16,40"), (9, "3,1000"), (1, "57,64"), (0, "16,3"), (4, "8,8"), (8, "12,7"),
]


@pytest.mark.parametrize("tile,sk", SK_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", [
    ("abij=acik*bkcj", dict(a=40, b=40, c=40, i=12, j=12, k=12)),
    ("ajbi=kcia*cjkb", dict(a=18, b=9, c=12, i=16, j=24, k=6)),
])
def test_stream_k_split(tile, sk, dtype, spec, ext, monkeypatch):
    """Forced stream-K splits of the gather kernel: partial tiles summed by
    the fixup kernel must match the oracle (bit-exact on integer inputs)."""
    if dtype == "f32" and tile in (7, 8, 9):
        pytest.skip("FP64-only tile")
    monkeypatch.setenv("COMET_GETT_TILE", str(tile))
    monkeypatch.setenv("COMET_GETT_SK", sk)
    check(spec, ext, dtype, seed=900 + tile, kind="integer", alpha=1.0, beta=1.0)
    check(spec, ext, dtype, seed=920 + tile, alpha=-0.75, beta=0.5)
    check(spec, ext, dtype, seed=940 + tile, alpha=1.5, beta=0.0, path="gett")


def test_stream_k_plan_describes_split(monkeypatch):
    monkeypatch.setenv("COMET_GETT_TILE", "3")
    monkeypatch.setenv("COMET_GETT_SK", "9,5")
    A = torch.zeros((40, 40, 12, 12), dtype=torch.float64, device="cuda")
    B = torch.zeros((40, 12, 40, 12), dtype=torch.float64, device="cuda")
    p = comet.Plan("abij=acik*bkcj", A, B, path="gett")
    d = p.describe()
    assert d["tile"] == 3 and d["sk_tiles"] == 9 and d["sk_blocks"] == 5
    assert p.workspace_bytes >= 2 * 5 * 128 * 128 * 8


def test_stream_k_is_deterministic(monkeypatch):
    """The fixup sums the pieces in a fixed order: repeated runs agree bit for bit."""
    monkeypatch.setenv("COMET_GETT_TILE", "3")
    monkeypatch.setenv("COMET_GETT_SK", "16,40")
    spec, ext = "abij=acik*bkcj", dict(a=40, b=40, c=40, i=12, j=12, k=12)
    A, B, C0 = inputs(spec, ext, 77, kind="uniform", beta=True)
    first = run(spec, A, B, C0, 1.0, 0.5, "f64")
    for _ in range(3):
        assert np.array_equal(run(spec, A, B, C0, 1.0, 0.5, "f64"), first)


PERSIST_CASES = [(3, "4"), (3, "1000"), (1, "5"), (0, "7"), (4, "2"), (5, "3"), (8, "3"), (2, "6")]


@pytest.mark.parametrize("tile,grid", PERSIST_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", [
    ("abcijk=daij*bcdk", dict(a=5, b=6, c=7, d=9, i=4, j=6, k=8)),     # K = 9: one step per tile
    ("abij=acik*bkcj", dict(a=20, b=18, c=6, i=9, j=8, k=6)),         # K = 36: two or three steps
    ("ajbi=kcia*cjkb", dict(a=18, b=9, c=12, i=16, j=24, k=6)),       # A m-contiguous, K = 72
])
def test_persistent_schedule(tile, grid, dtype, spec, ext, monkeypatch):
    """The persistent kernel (few workgroups walking many tiles, next tile's
    loads overlapped with the current tile's epilogue) against the oracle."""
    if dtype == "f32" and tile in (7, 8, 9):
        pytest.skip("FP64-only tile")
    monkeypatch.setenv("COMET_GETT_TILE", str(tile))
    monkeypatch.setenv("COMET_GETT_PERSIST", grid)
    check(spec, ext, dtype, seed=960 + tile, kind="integer", alpha=1.0, beta=1.0)
    check(spec, ext, dtype, seed=980 + tile, alpha=-0.75, beta=0.5)


def test_latency_bound_problems_spread_the_summation():
    """Fewer 64 x 64 tiles than one round of workgroups (the all-16
    contraction): tile 1 with its summation cut into stream-K pieces, and the
    result equals the oracle's."""
    spec, ext = CONFIG_SMALL[0]
    A, B, _ = inputs(spec, ext, 990)
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    d = comet.Plan(spec, Ad, Bd).describe()
    assert d["tile"] == 1 and d["sk_tiles"] == 16 and d["sk_blocks"] > d["sk_tiles"]
    print_case("latency-bound schedule")
    got = to_np(comet.contract(spec, Ad, Bd))
    assert oracle.relerr(got, oracle.contract(spec, A, B)) <= 1e-12


def test_persistent_only_on_request(monkeypatch):
    """The whole-tile kernel is the default for short summations too; the
    persistent schedule runs when COMET_GETT_PERSIST asks for it."""
    A = torch.zeros((32, 32, 16, 16), dtype=torch.float64, device="cuda")
    B = torch.zeros((32, 32, 32, 16), dtype=torch.float64, device="cuda")
    d = comet.Plan("abcijk=daij*bcdk", A, B).describe()
    assert d["persist"] == 0 and d["sk_tiles"] == 0
    monkeypatch.setenv("COMET_GETT_PERSIST", "256")
    d = comet.Plan("abcijk=daij*bcdk", A, B).describe()
    assert d["persist"] == 256


def test_contract_plan_cache_is_bounded():
    """comet_contract keeps at most 1024 plans per device: the 1025th distinct
    problem empties the cache, and every call before and after it (including
    a problem planned again after the reset) gives the exact result."""
    print_case("plan cache bound", "ij=ik*kj", "i = 1..1030")
    k, j = 5, 3
    B = synth.integers(31, (k, j))
    Bd = torch_dev(B, torch.float64)
    As = {}
    for i in list(range(1, 1031)) + [1, 2, 1030]:
        if i not in As:
            As[i] = synth.integers(1000 + i, (i, k))
        out = comet.contract("ij=ik*kj", torch_dev(As[i], torch.float64), Bd)
        if i % 97 == 1 or i >= 1020 or i <= 2:
            torch.cuda.synchronize()
            ref = oracle.contract("ij=ik*kj", As[i], B)
            assert np.array_equal(to_np(out), ref), "i = %d" % i
    torch.cuda.synchronize()


@pytest.mark.parametrize("spec,dtype,compute", [
    ("ij=ik*kj", "f32", "default"),
    ("ji=ik*kj", "f32", "default"),
    ("ij=ik*kj", "f64", "split_int8"),
    ("ji=ik*kj", "f64", "split_bf16x3"),
])
def test_output_beyond_2_31_elements(spec, dtype, compute):
    """C with 49152 x 49152 elements (2.4e9 > 2^31; 9.7 GB in FP32, 19.3 GB
    in FP64): every output address needs 64 bits.  Integer inputs, exact in
    every mode, so sampled outputs match the oracle bit for bit; all-ones
    inputs give K everywhere, which checks that every element up to the last
    one is written."""
    n, k = 49152, 16
    print_case("output beyond 2^31", spec, dtype, compute, n, k)
    A = synth.integers(71, (n, k))
    B = synth.integers(72, (k, n))
    Ad, Bd = torch_dev(A, tdt(dtype)), torch_dev(B, tdt(dtype))
    C = comet.contract(spec, Ad, Bd, compute=compute)
    torch.cuda.synchronize()
    assert C.numel() > (1 << 31)
    pts = sample_points(tuple(C.shape), 4000, 9)
    g = C[tuple(torch.from_numpy(pts).cuda().T)].cpu().numpy()
    ref = oracle.contract_points(spec, A, B, pts)
    assert np.array_equal(g, ref)
    del C
    C1 = comet.contract(spec, torch.ones_like(Ad), torch.ones_like(Bd), compute=compute)
    torch.cuda.synchronize()
    assert bool((C1 == float(k)).all())
    del C1
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operands_beyond_2_31_elements(dtype):
    """A and B with 64 x (2^25 + 8) elements each (2.1e9 > 2^31): operand
    addresses need 64 bits, and the single 64 x 64 output tile sums 2^21 + 1
    steps, the last one ragged.  A comb operand (1 where k mod 64 equals the
    row, else 0) times all-ones gives, in closed form, K // 64 plus one for
    the first K mod 64 rows -- exact in both precisions."""
    m, k = 64, (1 << 25) + 8
    t = tdt(dtype)
    print_case("operands beyond 2^31", dtype, m, k)
    kmod = torch.arange(k, device="cuda") % 64
    idx = torch.arange(m, device="cuda")
    want = torch.full((m,), float(k // 64), dtype=torch.float64, device="cuda") + (idx < k % 64).double()
    A = (kmod[None, :] == idx[:, None]).to(t)
    B = torch.ones((k, m), dtype=t, device="cuda")
    assert A.numel() > (1 << 31)
    C = comet.contract("ij=ik*kj", A, B)
    torch.cuda.synchronize()
    assert torch.equal(C.double(), want[:, None].expand(m, m))
    del A, B, C
    A = torch.ones((m, k), dtype=t, device="cuda")
    B = (kmod[:, None] == idx[None, :]).to(t)
    C = comet.contract("ij=ik*kj", A, B)
    torch.cuda.synchronize()
    assert torch.equal(C.double(), want[None, :].expand(m, m))
    del A, B, C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,compute", [("f64", "default"), ("f32", "default"), ("f64", "split_int8"),
                                           ("f64", "split_bf16x3"), ("f64", "ttgt")])
def test_broadcast_operands(dtype, compute):
    """Stride-0 (broadcast) operands: A constant along the summation label k,
    B constant along the free label b.  The oracle gets the materialized
    arrays."""
    ext = dict(a=21, b=19, c=23, i=13, j=11, k=9)
    spec = "abij=acik*bkcj"
    print_case("broadcast operands", dtype, compute)
    t = tdt(dtype)
    a0 = synth.uniform(801, (21, 23, 13, 1))
    b0 = synth.uniform(802, (1, 9, 23, 11))
    c0 = synth.uniform(803, shape_of("abij", ext))
    cast = np.float32 if dtype == "f32" else np.float64
    A = np.ascontiguousarray(np.broadcast_to(a0, shape_of("acik", ext))).astype(cast)
    B = np.ascontiguousarray(np.broadcast_to(b0, shape_of("bkcj", ext))).astype(cast)
    C0 = c0.astype(cast)
    Ad = torch_dev(a0, t).expand(*shape_of("acik", ext))
    Bd = torch_dev(b0, t).expand(*shape_of("bkcj", ext))
    assert Ad.stride()[3] == 0 and Bd.stride()[0] == 0
    Cd = torch_dev(C0, t)
    if compute == "ttgt":
        plan = comet.Plan(spec, Ad, Bd, Cd, compute="f64", path="ttgt")
        plan(Ad, Bd, Cd, alpha=0.5, beta=-1.0)
        mode = "f64"
    else:
        comet.contract(spec, Ad, Bd, Cd, alpha=0.5, beta=-1.0, compute=compute)
        mode = dtype if compute == "default" else compute
    torch.cuda.synchronize()
    ref = oracle.contract(spec, A, B, C0, alpha=0.5, beta=-1.0)
    err = oracle.relerr(to_np(Cd), ref)
    assert err <= dict(TOL, split_int8=1e-9)[mode], "relerr %.3e" % err


# operands whose unit-stride labels are different summation labels: only one
# of them can read 16-byte vectors along the fused K order, so the plan takes
# tile 1's element-load variant
ELEMENT_LOAD_CASES = [
    ("ia=ind*adn", dict(i=70, a=45, n=19, d=23)),
    ("ia=dn*inad", dict(d=40, n=24, i=9, a=33)),     # one output row per i: GEMV-like
]


@pytest.mark.parametrize("sk", [None, "3,7", "2,200"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", ELEMENT_LOAD_CASES)
def test_stream_k_element_load_variants(spec, ext, dtype, sk, monkeypatch):
    """Stream-K splits of tile 1's element-load variants (planned, and forced
    over tile boundaries and with more workgroups than steps) against the
    oracle, bit-exact on integer inputs."""
    if sk is not None:
        monkeypatch.setenv("COMET_GETT_TILE", "1")
        monkeypatch.setenv("COMET_GETT_SK", sk)
    check(spec, ext, dtype, seed=960, kind="integer", alpha=1.0, beta=1.0)
    check(spec, ext, dtype, seed=961, alpha=-0.5, beta=0.25)


def test_gemv_like_contraction_is_split(monkeypatch):
    """A contraction with one output row and a long summation: the
    matrix-vector kernel by default; with it switched off (COMET_GEMV=0) the
    gather path spreads the summation over the CUs by stream-K."""
    A = torch.zeros((96, 32), dtype=torch.float64, device="cuda")
    B = torch.zeros((32, 32, 96, 96), dtype=torch.float64, device="cuda")
    d = comet.Plan("ia=dn*inad", A, B).describe()
    assert d["gemv"] == 2 and d["gemv_split"] > 1
    monkeypatch.setenv("COMET_GEMV", "0")
    d = comet.Plan("ia=dn*inad", A, B).describe()
    assert d["gemv"] == 0 and d["tile"] == 1 and d["sk_tiles"] > 0 and d["sk_blocks"] > d["sk_tiles"]


def test_large_element_load_problem_goes_through_ttgt():
    """Operands whose unit strides lie on different summation labels can only
    be gathered by tile 1's element-load kernel; from 2^28 multiply-adds the
    planner permutes them instead (TTGT).  Sampled outputs match the oracle."""
    spec = "cmia=cdmn*inad"
    ext = dict(c=64, m=16, i=16, a=64, d=64, n=16)
    print_case("element-load problem via TTGT", spec, ext)
    A = synth.uniform(971, shape_of("cdmn", ext))
    B = synth.uniform(972, shape_of("inad", ext))
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    d = comet.Plan(spec, Ad, Bd).describe()
    assert d["path"] == "ttgt"
    C = comet.contract(spec, Ad, Bd)
    torch.cuda.synchronize()
    pts = sample_points(tuple(C.shape), 2000, 11)
    g = C[tuple(torch.from_numpy(pts).cuda().T)].cpu().numpy()
    assert oracle.relerr(g, oracle.contract_points(spec, A, B, pts)) <= 1e-12
    # below the threshold the gather path stays
    small = dict(c=32, m=16, i=16, a=32, d=32, n=16)
    As = torch.zeros(shape_of("cdmn", small), dtype=torch.float64, device="cuda")
    Bs = torch.zeros(shape_of("inad", small), dtype=torch.float64, device="cuda")
    assert comet.Plan(spec, As, Bs).describe()["path"] == "gett"
