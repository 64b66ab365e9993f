"""Parity of the compensated split-precision modes against the FP64 oracle.

Bars (relative Frobenius error): aligned BF16 and aligned INT8 slices <= 1e-9
on FP64 storage; classic BF16x3 and FP16x2 <= 1e-5 (FP32-class accumulation); any
split mode on FP32 storage <= 1e-5 (rounding the output to FP32 alone costs
~3e-8).  Integer-valued inputs are reproduced bit for bit in every mode:
their slices and partial sums are exact.
"""
import numpy as np
import pytest

from gpu_common import inputs, oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

MODES = ["split_bf16", "split_bf16x3", "split_fp16x2", "split_int8"]
TOL64 = {"split_bf16": 1e-9, "split_bf16x3": 1e-5, "split_fp16x2": 1e-5, "split_int8": 1e-9}

CASES = [
    ("abij=acik*cbkj", dict(a=16, b=16, c=16, i=16, j=16, k=16)),
    ("abij=acik*bkcj", dict(a=40, b=40, c=40, i=12, j=12, k=12)),
    ("abcijk=daij*bcdk", dict(a=10, b=9, c=7, d=12, i=6, j=5, k=6)),
    ("abij=ijcd*cdab", dict(a=9, b=13, c=7, d=11, i=10, j=14)),
    ("ajbi=kcia*cjkb", dict(a=17, b=9, c=12, i=8, j=24, k=6)),
    ("abcd=aebf*dfce", dict(a=13, b=11, c=12, d=9, e=10, f=7)),
]


def run(spec, A, B, C0, alpha, beta, tdt, compute):
    Ad, Bd = torch_dev(A, tdt), torch_dev(B, tdt)
    Cd = torch_dev(C0, tdt) if C0 is not None else None
    out = comet.contract(spec, Ad, Bd, Cd, alpha=alpha, beta=beta, compute=compute)
    torch.cuda.synchronize()
    return to_np(out)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec,ext", CASES)
def test_split_fp64_storage(spec, ext, mode):
    print_case("split f64", spec, mode)
    A, B, C0 = inputs(spec, ext, 800, kind="normal", beta=True)
    got = run(spec, A, B, C0, 1.25, -0.5, torch.float64, mode)
    ref = oracle.contract(spec, A, B, C0, alpha=1.25, beta=-0.5)
    err = oracle.relerr(got, ref)
    assert err <= TOL64[mode], "relerr %.3e" % err
    # the product alone (beta = 0), so C0 cannot hide product errors
    got0 = run(spec, A, B, None, 1.0, 0.0, torch.float64, mode)
    err0 = oracle.relerr(got0, oracle.contract(spec, A, B))
    assert err0 <= TOL64[mode], "relerr (beta=0) %.3e" % err0


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec,ext", CASES[:3])
def test_split_fp32_storage(spec, ext, mode):
    print_case("split f32", spec, mode)
    A, B, C0 = inputs(spec, ext, 810, beta=True)
    A32, B32, C32 = A.astype(np.float32), B.astype(np.float32), C0.astype(np.float32)
    got = run(spec, A32, B32, C32, 1.0, 1.0, torch.float32, mode)
    ref = oracle.contract(spec, A32, B32, C32, alpha=1.0, beta=1.0)
    assert oracle.relerr(got, ref) <= 1e-5


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec,ext", CASES)
def test_split_integer_inputs_bitwise(spec, ext, mode):
    print_case("split int", spec, mode)
    A, B, C0 = inputs(spec, ext, 820, kind="integer", beta=True)
    got = run(spec, A, B, C0, 1.0, 1.0, torch.float64, mode)
    assert np.array_equal(got, oracle.contract(spec, A, B, C0, alpha=1.0, beta=1.0))


def test_split_slices_control_the_error():
    spec, ext = CASES[1]
    A, B, _ = inputs(spec, ext, 830, kind="normal")
    ref = oracle.contract(spec, A, B)
    errs = {}
    try:
        for S in (3, 4, 5, 6):
            comet.set_split_slices(S)
            print_case("slices", S)
            errs[S] = oracle.relerr(run(spec, A, B, None, 1.0, 0.0, torch.float64, "split_bf16"), ref)
    finally:
        comet.set_split_slices(5)
    # more slices, less truncation error, down to the floor set by the FP32
    # accumulator shared by the pairs with p + q >= 2 (rounding 2^-24 on terms
    # 2^-16 below the leading ones: ~1e-11 relative)
    assert errs[3] > errs[4] > errs[5] >= errs[6] * 0.9
    assert errs[5] <= 1e-9 and errs[6] <= 1e-10


def test_split_zero_rows_and_tiny_values():
    """All-zero rows (exponent sentinel) and widely scaled rows."""
    spec = "ij=ik*kj"
    A = synth.normal(840, (70, 50))
    B = synth.normal(841, (50, 90))
    A[3, :] = 0.0
    B[:, 7] = 0.0
    A[5, :] *= 1e-200
    B[:, 9] *= 1e150
    print_case("split zero rows")
    for mode in MODES:
        got = run(spec, A, B, None, 1.0, 0.0, torch.float64, mode)
        ref = oracle.contract(spec, A, B)
        assert np.all(got[3, :] == 0.0) and np.all(got[:, 7] == 0.0)
        # row-wise relative error, so the scaled rows are judged on their own
        row = np.abs(got - ref).max(axis=1) / np.maximum(np.abs(ref).max(axis=1), 1e-300)
        assert row[5] <= TOL64[mode] * 100
        assert oracle.relerr(np.delete(got, [5], 0), np.delete(ref, [5], 0)) <= TOL64[mode] * 10


def config2_inputs():
    V, O = 96, 32
    ext = dict(a=V, b=V, c=V, i=O, j=O, k=O)
    A = synth.decayed_normal(synth.config_seed(2, "A"), "acik", shape_of("acik", ext), "abc", "ijk")
    B = synth.decayed_normal(synth.config_seed(2, "B"), "bkcj", shape_of("bkcj", ext), "abc", "ijk")
    C0 = synth.decayed_normal(synth.config_seed(2, "C0"), "abij", shape_of("abij", ext), "abc", "ijk")
    return ext, A, B, C0


@pytest.mark.parametrize("mode", MODES)
def test_split_config2_full_size_sampled(mode):
    spec = "abij=acik*bkcj"
    ext, A, B, C0 = config2_inputs()
    print_case("split config2", mode)
    rng = np.random.default_rng(5)
    pts = np.stack([rng.integers(0, n, 3000) for n in shape_of("abij", ext)], axis=1)
    got0 = run(spec, A, B, None, 1.0, 0.0, torch.float64, mode)
    ref0 = oracle.contract_points(spec, A, B, pts)
    err = oracle.relerr(got0[tuple(pts.T)], ref0)
    assert err <= TOL64[mode], "relerr %.3e" % err


@pytest.mark.parametrize("mode", MODES)
def test_split_config3_full_size_sampled(mode):
    spec = "abcijk=daij*bcdk"
    ext = dict(a=32, b=32, c=32, d=32, i=16, j=16, k=16)
    A = synth.uniform(synth.config_seed(3, "A"), shape_of("daij", ext))
    B = synth.uniform(synth.config_seed(3, "B"), shape_of("bcdk", ext))
    print_case("split config3", mode)
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    C = comet.contract(spec, Ad, Bd, compute=mode)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    pts = np.stack([rng.integers(0, n, 4000) for n in C.shape], axis=1)
    g = C[tuple(torch.from_numpy(pts).cuda().T)].cpu().numpy()
    assert oracle.relerr(g, oracle.contract_points(spec, A, B, pts)) <= TOL64[mode]
    del C


def test_int8_slices_control_the_error():
    """INT8 slices accumulate exactly, so the error keeps falling with S."""
    spec, ext = CASES[1]
    A, B, _ = inputs(spec, ext, 850, kind="normal")
    ref = oracle.contract(spec, A, B)
    errs = {}
    try:
        for S in (3, 4, 5, 6, 7, 8):
            comet.set_int8_slices(S)
            print_case("int8 slices", S)
            errs[S] = oracle.relerr(run(spec, A, B, None, 1.0, 0.0, torch.float64, "split_int8"), ref)
    finally:
        comet.set_int8_slices(6)
    for S in (3, 4, 5, 6, 7):
        assert errs[S] > errs[S + 1], errs
    assert errs[6] <= 1e-9 and errs[8] <= 1e-13, errs


def test_int8_long_summation_is_chunked():
    """A summation longer than one launch's exact int32 range (8192 indices)."""
    A = synth.normal(860, (96, 20000))
    B = synth.normal(861, (20000, 80))
    C0 = synth.normal(862, (96, 80))
    print_case("int8 long K")
    got = run("ij=ik*kj", A, B, C0, 1.0, 1.0, torch.float64, "split_int8")
    assert oracle.relerr(got, oracle.contract("ij=ik*kj", A, B, C0, beta=1.0)) <= 1e-9


@pytest.mark.parametrize("mode", ["split_bf16x3", "split_fp16x2"])
@pytest.mark.parametrize("spec,ext", CASES)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_split_large_tile_forced(spec, ext, mode, storage, monkeypatch):
    """The 192 x 192 slice-pair kernel on ragged problems (operands padded to
    multiples of 192): same bars, integer inputs bit for bit."""
    monkeypatch.setenv("COMET_SPLIT_TILE", "1")
    monkeypatch.setenv("COMET_FUSED3", "0")   # FP32 BF16x3 through the slicer too
    tdt = torch.float64 if storage == "f64" else torch.float32
    cast = np.float64 if storage == "f64" else np.float32
    print_case("split large tile", spec, mode, storage)
    A, B, C0 = inputs(spec, ext, 830, kind="normal", beta=True)
    A, B, C0 = A.astype(cast), B.astype(cast), C0.astype(cast)
    got = run(spec, A, B, C0, 1.25, -0.5, tdt, mode)
    ref = oracle.contract(spec, A, B, C0, alpha=1.25, beta=-0.5)
    assert oracle.relerr(got, ref) <= 1e-5
    Ai, Bi, _ = inputs(spec, ext, 831, kind="integer", beta=False)
    gi = run(spec, Ai, Bi, None, 1.0, 0.0, tdt, mode)
    assert np.array_equal(gi, oracle.contract(spec, Ai.astype(cast), Bi.astype(cast)))


def test_split_large_tile_is_chosen_for_large_products():
    V, O = 96, 32
    A = torch.zeros((V, V, O, O), dtype=torch.float64, device="cuda")
    B = torch.zeros((V, O, V, O), dtype=torch.float64, device="cuda")
    d = comet.Plan("abij=acik*bkcj", A, B, compute="split_bf16x3").describe()
    assert d.get("split_tile") == 1


WIDE_CASES = [
    # ragged M and N (not multiples of 128 and 192), K = 300: ten 32-index
    # stages, two groups of four and a tail of two
    ("ij=ik*kj", dict(i=200, j=250, k=300)),
    ("abij=acik*bkcj", dict(a=40, b=40, c=40, i=12, j=12, k=12)),
    ("abcd=aebf*dfce", dict(a=13, b=11, c=12, d=9, e=10, f=7)),
]


@pytest.mark.parametrize("S", [3, 4, 5, 6])
@pytest.mark.parametrize("spec,ext", WIDE_CASES)
def test_split_wide_tile_forced(spec, ext, S, monkeypatch):
    """The 128 x 96 aligned slice-pair kernel (COMET_SPLIT_TILE=2) on ragged
    problems: FP64 storage as close to the oracle as the 128 x 64 tile (the
    same slice pairs, accumulators and fold length) and within the aligned
    bar at S >= 5, FP32 storage within 1e-5, integer inputs bit for bit, and
    all-zero rows exact.  Six slices do not fit its LDS: the plan falls back
    to the 128 x 64 tile."""
    A, B, C0 = inputs(spec, ext, 870, kind="normal", beta=True)
    A[(0,) * A.ndim] = 0.0
    A[(1,) + (slice(None),) * (A.ndim - 1)] = 0.0   # a zero slab: zero rows of the matrix view
    ref = oracle.contract(spec, A, B, C0, alpha=1.25, beta=-0.5)
    try:
        comet.set_split_slices(S)
        monkeypatch.setenv("COMET_SPLIT_TILE", "0")
        err0 = oracle.relerr(run(spec, A, B, C0, 1.25, -0.5, torch.float64, "split_bf16"), ref)
        monkeypatch.setenv("COMET_SPLIT_TILE", "2")
        d = comet.Plan(spec, torch_dev(A, torch.float64), torch_dev(B, torch.float64),
                       compute="split_bf16").describe()
        assert d["split_tile"] == (2 if S <= 5 else 0), d
        print_case("split wide tile", spec, S)
        got = run(spec, A, B, C0, 1.25, -0.5, torch.float64, "split_bf16")
        assert np.all(got[oracle.contract(spec, A, B) == 0.0] == (-0.5 * C0)[oracle.contract(spec, A, B) == 0.0])
        err = oracle.relerr(got, ref)
        assert err <= 2.0 * err0 + 1e-15, "relerr %.3e against %.3e on the 128 x 64 tile" % (err, err0)
        assert S < 5 or err <= 1e-9, "relerr %.3e" % err
        A32, B32 = A.astype(np.float32), B.astype(np.float32)
        g32 = run(spec, A32, B32, None, 1.0, 0.0, torch.float32, "split_bf16")
        assert oracle.relerr(g32, oracle.contract(spec, A32, B32)) <= 1e-5
        Ai, Bi, Ci = inputs(spec, ext, 871, kind="integer", beta=True)
        gi = run(spec, Ai, Bi, Ci, 1.0, 1.0, torch.float64, "split_bf16")
        assert np.array_equal(gi, oracle.contract(spec, Ai, Bi, Ci, alpha=1.0, beta=1.0))
    finally:
        comet.set_split_slices(5)


def test_split_wide_tile_is_chosen_for_large_aligned_products():
    V, O = 96, 32
    A = torch.zeros((V, V, O, O), dtype=torch.float64, device="cuda")
    B = torch.zeros((V, O, V, O), dtype=torch.float64, device="cuda")
    assert comet.Plan("abij=acik*bkcj", A, B, compute="split_bf16").describe().get("split_tile") == 2
    small = torch.zeros((300, 300), dtype=torch.float64, device="cuda")
    assert comet.Plan("ij=ik*kj", small, small, compute="split_bf16").describe().get("split_tile") == 0


@pytest.mark.parametrize("fused", ["1", "0"])
@pytest.mark.parametrize("spec,ext", CASES)
def test_fp32_bf16x3_fused_and_sliced_paths(spec, ext, fused, monkeypatch):
    """FP32 storage in BF16x3: the fused kernel (operands split in the loader)
    and the slicer + slice-pair product, each against the oracle."""
    monkeypatch.setenv("COMET_FUSED3", fused)
    print_case("fp32 bf16x3", spec, "fused" if fused == "1" else "sliced")
    A, B, C0 = inputs(spec, ext, 840, beta=True)
    A32, B32, C32 = A.astype(np.float32), B.astype(np.float32), C0.astype(np.float32)
    Ad, Bd = torch_dev(A32, torch.float32), torch_dev(B32, torch.float32)
    assert comet.Plan(spec, Ad, Bd, compute="split_bf16x3").describe()["fused3"] is (fused == "1")
    got = run(spec, A32, B32, C32, 1.5, -1.0, torch.float32, "split_bf16x3")
    assert oracle.relerr(got, oracle.contract(spec, A32, B32, C32, alpha=1.5, beta=-1.0)) <= 1e-5


def test_fp32_bf16x3_path_follows_the_product_size():
    small = torch.zeros((256, 256), dtype=torch.float32, device="cuda")
    assert comet.Plan("ij=ik*kj", small, small, compute="split_bf16x3").describe()["fused3"] is True
    big_a = torch.zeros((1400, 1400), dtype=torch.float32, device="cuda")
    d = comet.Plan("ij=ik*kj", big_a, big_a, compute="split_bf16x3").describe()
    assert d["fused3"] is False and "split_tile" in d


def test_fp32_bf16x3_sliced_path_at_size_sampled():
    """Above the size threshold (1400^3 multiply-adds) on sampled outputs."""
    n = 1400
    A = synth.uniform(850, (n, n)).astype(np.float32)
    B = synth.uniform(851, (n, n)).astype(np.float32)
    print_case("fp32 bf16x3 sliced 1400^3")
    got = run("ij=ik*kj", A, B, None, 1.0, 0.0, torch.float32, "split_bf16x3")
    rng = np.random.default_rng(852)
    pts = np.stack([rng.integers(0, n, 2000), rng.integers(0, n, 2000)], axis=1)
    ref = oracle.contract_points("ij=ik*kj", A, B, pts)
    assert oracle.relerr(got[tuple(pts.T)], ref) <= 1e-5


@pytest.mark.parametrize("mode", MODES)
def test_split_degenerate(mode):
    """The split modes on the degenerate problems: an empty summation
    (C = beta * C), an empty output, a full contraction to a scalar, alpha = 0
    with NaN in A (A and B unread), and extent-1 labels everywhere."""
    print_case("split degenerate", mode)
    f64 = torch.float64
    C0 = synth.uniform(41, (5, 7))
    C = torch_dev(C0, f64)
    comet.contract("ij=ik*kj", torch.zeros((5, 0), dtype=f64, device="cuda"),
                   torch.zeros((0, 7), dtype=f64, device="cuda"), C, beta=3.0, compute=mode)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), 3.0 * C0)
    C = comet.contract("ij=ik*kj", torch.zeros((0, 4), dtype=f64, device="cuda"),
                       torch.ones((4, 3), dtype=f64, device="cuda"), compute=mode)
    assert C.shape == (0, 3)
    Ai = synth.integers(42, (37, 41))
    Bi = synth.integers(43, (41, 37))
    C = comet.contract("=ab*ba", torch_dev(Ai, f64), torch_dev(Bi, f64), compute=mode)
    torch.cuda.synchronize()
    assert float(C.item()) == float(np.sum(Ai * Bi.T))
    A = torch.full((6, 4), float("nan"), dtype=f64, device="cuda")
    B = torch_dev(synth.uniform(44, (4, 5)), f64)
    C0 = synth.uniform(45, (6, 5))
    C = torch_dev(C0, f64)
    comet.contract("ij=ik*kj", A, B, C, alpha=0.0, beta=-2.0, compute=mode)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), -2.0 * C0)
    ext = dict(a=1, b=1, c=1, i=1, j=1, k=1)
    A, B, _ = inputs("abij=acik*cbkj", ext, 46, kind="integer")
    C = comet.contract("abij=acik*cbkj", torch_dev(A, f64), torch_dev(B, f64), compute=mode)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), oracle.contract("abij=acik*cbkj", A, B))
