"""Batch labels (a label in C, A and B: indexed alike, not summed) and
stepped index ranges as views, on the HIP path, against the CPU FP64 oracle.

Bars as in the other parity tests: relative Frobenius error <= 1e-12 (FP64
arithmetic) or <= 1e-5 (FP32 and the FP32-level split modes), bit-exact for
integer-valued inputs.
"""
import numpy as np
import pytest

from gpu_common import TOL, inputs, oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

TOL_ALL = dict(TOL, split_int8=1e-9)


def tdt(name):
    return torch.float64 if name == "f64" else torch.float32


def check(spec, ext, dtype="f64", seed=0, kind="uniform", alpha=1.0, beta=0.0, compute="default"):
    print_case("batch labels", spec, ext, dtype, kind, alpha, beta, compute)
    A, B, C0 = inputs(spec, ext, seed, kind=kind, beta=True)
    cast = np.float32 if dtype == "f32" else np.float64
    A, B, C0 = A.astype(cast), B.astype(cast), C0.astype(cast)
    Ad, Bd, Cd = torch_dev(A, tdt(dtype)), torch_dev(B, tdt(dtype)), torch_dev(C0, tdt(dtype))
    comet.contract(spec, Ad, Bd, Cd, alpha=alpha, beta=beta, compute=compute)
    torch.cuda.synchronize()
    got = to_np(Cd)
    ref = oracle.contract(spec, A, B, C0, alpha=alpha, beta=beta)
    if kind == "integer":
        assert np.array_equal(got, ref)
    else:
        mode = dtype if compute == "default" else compute
        err = oracle.relerr(got, ref)
        assert err <= TOL_ALL[mode], "relerr %.3e" % err
    return got


CASES = [
    # batched matrix products, several tiles per entry plus a ragged tail
    ("bij=bik*bkj", dict(b=5, i=70, j=67, k=45)),
    # batch label innermost in C, permuted operands
    ("ibj=kbi*jbk", dict(b=3, i=33, j=70, k=29)),
    # two batch labels, not adjacent, and a free label of each kind
    ("xaiy=xyk*kyia", dict(x=3, y=4, a=9, i=17, k=11)),
    # many small entries: more workgroups from the batch than from the tiles
    ("bij=bik*bkj", dict(b=700, i=9, j=7, k=5)),
    # every label a batch label: the elementwise product
    ("ijk=ijk*ijk", dict(i=13, j=11, k=17)),
    # a batch of dot products
    ("b=bk*bk", dict(b=37, k=130)),
    # batch label with an outer product per entry
    ("bij=bi*bj", dict(b=6, i=40, j=66)),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_batch_labels_match_oracle(case, dtype):
    spec, ext = CASES[case]
    check(spec, ext, dtype, seed=100 + case, alpha=1.5, beta=-0.5)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_batch_labels_integer_exact(case):
    spec, ext = CASES[case]
    check(spec, ext, "f64", seed=200 + case, kind="integer", alpha=1.0, beta=1.0)


@pytest.mark.parametrize("tile", ["1", "3"])
def test_batch_labels_each_tile(tile, monkeypatch):
    monkeypatch.setenv("COMET_GETT_TILE", tile)
    check("bij=bik*bkj", dict(b=4, i=200, j=150, k=70), "f64", seed=301)
    check("ibj=kbi*jbk", dict(b=3, i=150, j=140, k=33), "f32", seed=302)


@pytest.mark.parametrize("compute", ["split_bf16", "split_bf16x3", "split_fp16x2", "split_int8"])
def test_batch_labels_split_modes(compute):
    """The split modes run one contraction per batch entry."""
    check("bij=bik*bkj", dict(b=3, i=40, j=35, k=50), "f64", seed=311, alpha=2.0, beta=1.0, compute=compute)


def test_batch_labels_fused_bf16x3_on_fp32():
    check("bij=bik*bkj", dict(b=4, i=70, j=66, k=40), "f32", seed=312, compute="split_bf16x3")


def test_batch_labels_unaligned_entries():
    """Odd batch strides: entries are not 16-byte aligned, so the element-load
    variants run."""
    ext = dict(b=5, i=21, j=19, k=13)
    A = synth.uniform(321, (5, 21 * 13 + 1))[:, :21 * 13].reshape(5, 21, 13)   # batch stride 274
    B = synth.uniform(322, (5, 13, 19))
    C0 = synth.uniform(323, (5, 21, 19))
    baseA = torch_dev(synth.uniform(321, (5, 21 * 13 + 1)), torch.float64)
    Ad = baseA[:, :21 * 13].unflatten(1, (21, 13))
    assert Ad.stride() == (274, 13, 1)
    Bd, Cd = torch_dev(B, torch.float64), torch_dev(C0, torch.float64)
    print_case("batch labels unaligned", ext)
    comet.contract("bij=bik*bkj", Ad, Bd, Cd, alpha=1.0, beta=1.0)
    torch.cuda.synchronize()
    ref = oracle.contract("bij=bik*bkj", to_np(Ad), B, C0, alpha=1.0, beta=1.0)
    assert oracle.relerr(to_np(Cd), ref) <= 1e-12


def test_batch_labels_alpha_zero_and_empty_sum():
    spec, ext = "bij=bik*bkj", dict(b=6, i=9, j=10, k=4)
    C0 = synth.uniform(331, (6, 9, 10))
    Ad = torch.full((6, 9, 4), float("nan"), dtype=torch.float64, device="cuda")
    Bd = torch.full((6, 4, 10), float("nan"), dtype=torch.float64, device="cuda")
    Cd = torch_dev(C0, torch.float64)
    print_case("batch labels alpha 0")
    comet.contract(spec, Ad, Bd, Cd, alpha=0.0, beta=-2.0)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(Cd), -2.0 * C0)
    # K = 0: C = beta * C over every batch entry
    Ad = torch.empty((6, 9, 0), dtype=torch.float64, device="cuda")
    Bd = torch.empty((6, 0, 10), dtype=torch.float64, device="cuda")
    Cd = torch_dev(C0, torch.float64)
    comet.contract(spec, Ad, Bd, Cd, alpha=1.0, beta=0.5)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(Cd), 0.5 * C0)
    # empty batch: nothing happens
    Ad = torch.empty((0, 9, 4), dtype=torch.float64, device="cuda")
    Bd = torch.empty((0, 4, 10), dtype=torch.float64, device="cuda")
    Cd = torch.empty((0, 9, 10), dtype=torch.float64, device="cuda")
    comet.contract(spec, Ad, Bd, Cd)
    torch.cuda.synchronize()


def test_batch_labels_strided_C_slice_untouched_elsewhere():
    spec = "bij=bik*bkj"
    A = synth.uniform(341, (4, 30, 12))
    B = synth.uniform(342, (4, 12, 28))
    base_C = synth.uniform(343, (9, 33, 31))
    Cfull = torch_dev(base_C, torch.float64)
    Cd = Cfull[1:9:2, 2:32, 1:29]
    print_case("batch labels C slice")
    comet.contract(spec, torch_dev(A, torch.float64), torch_dev(B, torch.float64), Cd, alpha=1.0, beta=1.0)
    torch.cuda.synchronize()
    ref = oracle.contract(spec, A, B, base_C[1:9:2, 2:32, 1:29], alpha=1.0, beta=1.0)
    assert oracle.relerr(to_np(Cd), ref) <= 1e-12
    mask = np.ones(base_C.shape, bool)
    mask[1:9:2, 2:32, 1:29] = False
    assert np.array_equal(to_np(Cfull)[mask], base_C[mask])


def test_batch_labels_plan_and_determinism():
    spec, ext = "bij=bik*bkj", dict(b=8, i=100, j=90, k=64)
    A, B, _ = inputs(spec, ext, 351)
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    C1 = torch.empty((8, 100, 90), dtype=torch.float64, device="cuda")
    plan = comet.Plan(spec, Ad, Bd, C1)
    d = plan.describe()
    assert d["nb"] == 8 and d["sk_tiles"] == 0 and d["persist"] == 0 and d["tile"] in (1, 3)
    print_case("batch labels plan")
    plan(Ad, Bd, C1)
    C2 = torch.empty_like(C1)
    plan(Ad, Bd, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    assert oracle.relerr(to_np(C1), oracle.contract(spec, A, B)) <= 1e-12


def test_batch_api_with_batch_labels():
    """The batch API expands a problem with batch labels into one problem per
    entry, next to ordinary problems."""
    probs, refs = [], []
    specs = [("bij=bik*bkj", dict(b=5, i=40, j=33, k=20)), ("ij=ik*kj", dict(i=70, j=50, k=30)),
             ("ibj=kbi*jbk", dict(b=3, i=20, j=66, k=9)), ("bij=bik*bkj", dict(b=2, i=8, j=8, k=0))]
    for n, (spec, ext) in enumerate(specs):
        A, B, C0 = inputs(spec, ext, 360 + 10 * n, beta=True)
        probs.append(dict(spec=spec, A=torch_dev(A, torch.float64), B=torch_dev(B, torch.float64),
                          C=torch_dev(C0, torch.float64), alpha=1.25, beta=-1.0))
        refs.append(oracle.contract(spec, A, B, C0, alpha=1.25, beta=-1.0))
    print_case("batch api with batch labels")
    batch = comet.Batch(probs, dtype=torch.float64)
    batch()
    torch.cuda.synchronize()
    for pr, ref in zip(probs, refs):
        assert oracle.relerr(to_np(pr["C"]), ref) <= 1e-12


def test_batch_labels_backward():
    """dA and dB of a contraction with batch labels are contractions with
    batch labels too (the same kernels), against the oracle's gradient."""
    spec, ext = "ixj=kxi*jxk", dict(i=30, x=4, j=26, k=21)
    A, B, C0 = inputs(spec, ext, 371, beta=True)
    W = synth.uniform(374, shape_of("ixj", ext))
    print_case("batch labels backward")
    Ad = torch_dev(A, torch.float64).requires_grad_(True)
    Bd = torch_dev(B, torch.float64).requires_grad_(True)
    Cd = torch_dev(C0, torch.float64).requires_grad_(True)
    C = comet.contract_ad(spec, Ad, Bd, Cd, alpha=0.5, beta=2.0)
    (C * torch_dev(W, torch.float64)).sum().backward()
    torch.cuda.synchronize()
    dA, dB, dC0 = oracle.grad(spec, A, B, W, alpha=0.5, beta=2.0)
    assert oracle.relerr(to_np(Ad.grad), dA) <= 1e-12
    assert oracle.relerr(to_np(Bd.grad), dB) <= 1e-12
    assert np.array_equal(to_np(Cd.grad), dC0)


# --------------------------------------------------------------------------
# stepped index ranges [lo:hi:step] as views
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_stepped_ranges_as_views(dtype):
    """Each operand a view with steps > 1 along several labels (the base
    pointer at lo, strides multiplied by the step)."""
    spec = "abij=acik*bkcj"
    base_A = synth.uniform(401, (41, 50, 30, 33))
    base_B = synth.uniform(402, (37, 31, 46, 20))
    base_C = synth.uniform(403, (44, 40, 19, 25))
    # a = 20, c = 16, i = 10, k = 11, b = 18, j = 8
    A = base_A[1:41:2, 3:50:3, 0:30:3, 2:33:3]
    B = base_B[0:36:2, 1:23:2, 4:36:2, 1:17:2]
    C = base_C[2:42:2, 0:36:2, 0:19:2, 3:25:3]
    ext = dict(a=20, c=16, i=10, k=11, b=18, j=8)
    assert A.shape == shape_of("acik", ext) and B.shape == shape_of("bkcj", ext) and C.shape == shape_of("abij", ext)
    cast = np.float32 if dtype == "f32" else np.float64
    Afull, Bfull, Cfull = torch_dev(base_A, tdt(dtype)), torch_dev(base_B, tdt(dtype)), torch_dev(base_C, tdt(dtype))
    Ad = Afull[1:41:2, 3:50:3, 0:30:3, 2:33:3]
    Bd = Bfull[0:36:2, 1:23:2, 4:36:2, 1:17:2]
    Cd = Cfull[2:42:2, 0:36:2, 0:19:2, 3:25:3]
    print_case("stepped views", dtype)
    comet.contract(spec, Ad, Bd, Cd, alpha=-1.0, beta=0.5)
    torch.cuda.synchronize()
    ref = oracle.contract(spec, A.astype(cast), B.astype(cast), C.astype(cast), alpha=-1.0, beta=0.5)
    assert oracle.relerr(to_np(Cd), ref) <= TOL[dtype]
    mask = np.ones(base_C.shape, bool)
    mask[2:42:2, 0:36:2, 0:19:2, 3:25:3] = False
    assert np.array_equal(to_np(Cfull)[mask], base_C.astype(cast)[mask])


def test_stepped_views_with_batch_labels():
    spec = "bij=bik*bkj"
    base_A = synth.uniform(411, (12, 40, 30))
    base_B = synth.uniform(412, (12, 30, 50))
    A, B = base_A[::3, 1::2, ::2], base_B[::3, ::2, 3:48:3]
    Ad = torch_dev(base_A, torch.float64)[::3, 1::2, ::2]
    Bd = torch_dev(base_B, torch.float64)[::3, ::2, 3:48:3]
    print_case("stepped views with batch labels")
    Cd = comet.contract(spec, Ad, Bd)
    torch.cuda.synchronize()
    assert oracle.relerr(to_np(Cd), oracle.contract(spec, A, B)) <= 1e-12


@pytest.mark.parametrize("spec,ext", [
    ("bij=bik*bkj", dict(b=140001, i=3, j=2, k=5)),
    ("ijk=ijk*ijk", dict(i=300, j=301, k=2)),
])
def test_batch_labels_beyond_one_launch(spec, ext):
    """More batch entries than one launch's grid holds along y (65535): the
    entries run in several launches, each from its own first entry; integer
    inputs, bit-exact against the oracle."""
    check(spec, ext, dtype="f64", seed=17, kind="integer")
    check(spec, ext, dtype="f32", seed=18, kind="integer", beta=1.0)
