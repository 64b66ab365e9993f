"""The matrix-vector kernel (contractions whose vector operand has no free
label, so the product has one output row) against the oracle: both reading
orders of the matrix (along its free labels, along the summation), one slab
and many, ragged summation and output lengths, FP64 and FP32, beta = 0 (C
never read) and beta != 0, strided views, a dot product, determinism, and the
chain's matrix-vector steps at full size."""
import numpy as np
import pytest

from gpu_common import TOL, inputs, oracle, print_case, shape_of, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

DT = {"f64": torch.float64, "f32": torch.float32}
CAST = {"f64": np.float64, "f32": np.float32}

# spec, extents, the expected reading order (1: along the free labels of the
# matrix, 2: along the summation)
CASES = [
    ("dn=mc*cdmn", dict(c=96, d=96, m=32, n=32), 1),        # the chain's first step (K = J = 3072)
    ("ia=dn*inad", dict(d=96, n=32, i=32, a=96), 2),        # its second step
    ("dn=mc*cdmn", dict(c=7, d=5, m=3, n=13), 1),           # one slab, ragged everything
    ("ia=dn*inad", dict(d=9, n=5, i=3, a=7), 2),
    ("dn=mc*cdmn", dict(c=45, d=11, m=37, n=9), 1),          # K = 1665 in many slabs, J = 99
    ("ia=dn*inad", dict(d=131, n=17, i=5, a=3), 2),         # K = 2227 in many slabs, J = 15
    ("j=k*kj", dict(k=70000, j=3), 1),                      # a long summation, three outputs
    ("j=k*jk", dict(k=70000, j=5), 2),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext,order", CASES)
def test_gemv_matches_oracle(spec, ext, order, dtype):
    for kind, alpha, beta, seed in (("integer", 1.0, 1.0, 9101), ("uniform", -0.75, 0.5, 9111),
                                    ("uniform", 1.25, 0.0, 9121)):
        print_case("gemv", spec, ext, dtype, kind, beta)
        A, B, C0 = inputs(spec, ext, seed, kind=kind, beta=True)
        Ad, Bd, Cd = torch_dev(A, DT[dtype]), torch_dev(B, DT[dtype]), torch_dev(C0, DT[dtype])
        if beta == 0.0:
            Cd.fill_(float("nan"))       # beta = 0 never reads C
        plan = comet.Plan(spec, Ad, Bd, Cd)
        d = plan.describe()
        assert d["gemv"] == order and d["gemv_split"] >= 1, d
        plan(Ad, Bd, Cd, alpha=alpha, beta=beta)
        torch.cuda.synchronize()
        c = CAST[dtype]
        ref = oracle.contract(spec, A.astype(c), B.astype(c), C0.astype(c) if beta else None, alpha=alpha, beta=beta)
        got = to_np(Cd)
        if kind == "integer":
            assert np.array_equal(got, ref), "integer inputs must match bit for bit"
        else:
            assert oracle.relerr(got, ref) <= TOL[dtype]


def test_gemv_slab_counts():
    """The chain-sized steps cut the summation into several slabs (partial
    sums plus the fix-up); a summation of at most one slab with enough
    outputs writes C directly."""
    for spec, ext in (("dn=mc*cdmn", dict(c=96, d=96, m=32, n=32)), ("ia=dn*inad", dict(d=96, n=32, i=32, a=96))):
        c, a, b = oracle.split_spec(spec)
        A = torch.zeros(shape_of(a, ext), dtype=torch.float64, device="cuda")
        B = torch.zeros(shape_of(b, ext), dtype=torch.float64, device="cuda")
        d = comet.Plan(spec, A, B).describe()
        assert d["gemv_split"] > 1, d
    ext = dict(k=60, j=5000)
    A, B, _ = inputs("j=k*kj", ext, 9151)
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    d = comet.Plan("j=k*kj", Ad, Bd).describe()
    assert d["gemv"] == 1 and d["gemv_split"] == 1, d
    print_case("gemv one slab", ext)
    got = comet.contract("j=k*kj", Ad, Bd)
    assert oracle.relerr(to_np(got), oracle.contract("j=k*kj", A, B)) <= 1e-12


def test_gemv_strided_views_and_dot_product():
    """Operands and C as strided views (every offset table non-trivial), and
    a dot product (one output, one vector each side)."""
    spec = "ia=dn*inad"
    ext = dict(d=40, n=12, i=6, a=10)
    A, B, C0 = inputs(spec, ext, 9131, kind="integer", beta=True)
    Abig = torch_dev(np.zeros((80, 12)), torch.float64)
    Abig[::2].copy_(torch_dev(A, torch.float64))
    Bbig = torch_dev(np.zeros((6, 12, 10, 41)), torch.float64)
    Bbig[..., :40].copy_(torch_dev(B, torch.float64))
    Cbig = torch_dev(np.zeros((6, 20)), torch.float64)
    Cv = Cbig[:, ::2]
    Cv.copy_(torch_dev(C0, torch.float64))
    print_case("gemv strided", ext)
    plan = comet.Plan(spec, Abig[::2], Bbig[..., :40], Cv)
    assert plan.describe()["gemv"] > 0
    plan(Abig[::2], Bbig[..., :40], Cv, alpha=1.0, beta=-1.0)
    torch.cuda.synchronize()
    ref = oracle.contract(spec, A, B, C0, alpha=1.0, beta=-1.0)
    assert np.array_equal(to_np(Cv), ref)
    assert np.all(to_np(Cbig[:, 1::2]) == 0.0)    # untouched between the view's columns
    # a dot product
    x = torch_dev(np.arange(1, 2001, dtype=np.float64).reshape(40, 50) % 7 - 3, torch.float64)
    y = torch_dev(np.arange(2000, dtype=np.float64).reshape(40, 50) % 5 - 2, torch.float64)
    print_case("gemv dot")
    p = comet.Plan("=ab*ab", x, y)
    assert p.describe()["gemv"] > 0
    got = to_np(comet.contract("=ab*ab", x, y))
    assert got.shape == () and float(got) == float((to_np(x) * to_np(y)).sum())


def test_gemv_is_deterministic_and_can_be_switched_off(monkeypatch):
    """Partial sums are added in slab order: repeated runs agree bit for bit;
    COMET_GEMV=0 keeps the gather path, and both equal the oracle."""
    spec = "dn=mc*cdmn"
    ext = dict(c=96, d=96, m=32, n=32)
    A, B, _ = inputs(spec, ext, 9141)
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    print_case("gemv determinism")
    plan = comet.Plan(spec, Ad, Bd)
    assert plan.describe()["gemv"] == 1
    first = to_np(plan(Ad, Bd))
    for _ in range(3):
        assert np.array_equal(to_np(plan(Ad, Bd)), first)
    ref = oracle.contract(spec, A, B)
    assert oracle.relerr(first, ref) <= 1e-12
    monkeypatch.setenv("COMET_GEMV", "0")
    off = comet.Plan(spec, Ad, Bd)
    assert off.describe()["gemv"] == 0
    assert oracle.relerr(to_np(off(Ad, Bd)), ref) <= 1e-12
