"""Backward of the contraction: dA and dB are themselves permuted contractions
run by the same kernels, behind torch.autograd.Function.

Checked against the oracle's gradient (FP64 <= 1e-12, aligned BF16 and INT8
splits <= 1e-9, BF16x3 <= 1e-5),
against central finite differences of the GPU forward on a 12-extent copy of
the CCSD-like workload (h = 1e-6; the loss is bilinear, so the difference
quotient is exact up to rounding), and by the dot-product (adjoint) identity.
"""
import numpy as np
import pytest

from gpu_common import oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

SPEC = "abij=acik*bkcj"


def ccsd_inputs(V, O, seed):
    ext = dict(a=V, b=V, c=V, i=O, j=O, k=O)
    A = synth.decayed_normal(seed + 1, "acik", shape_of("acik", ext), "abc", "ijk")
    B = synth.decayed_normal(seed + 2, "bkcj", shape_of("bkcj", ext), "abc", "ijk")
    W = synth.uniform(seed + 4, shape_of("abij", ext))
    C0 = synth.decayed_normal(seed + 3, "abij", shape_of("abij", ext), "abc", "ijk")
    return ext, A, B, C0, W


@pytest.mark.parametrize("compute,tol", [("f64", 1e-12), ("split_bf16", 1e-9), ("split_int8", 1e-9),
                                         ("split_bf16x3", 1e-5)])
@pytest.mark.parametrize("V,O", [(12, 12), (40, 12)])
def test_backward_matches_oracle_gradient(compute, tol, V, O):
    ext, A, B, C0, W = ccsd_inputs(V, O, 900)
    print_case("backward", compute, V, O)
    Ad = torch_dev(A, torch.float64).requires_grad_(True)
    Bd = torch_dev(B, torch.float64).requires_grad_(True)
    Cd = torch_dev(C0, torch.float64).requires_grad_(True)
    Wd = torch_dev(W, torch.float64)
    C = comet.contract_ad(SPEC, Ad, Bd, Cd, alpha=0.75, beta=1.5, compute=compute)
    loss = (C * Wd).sum()
    loss.backward()
    torch.cuda.synchronize()
    dA, dB, dC0 = oracle.grad(SPEC, A, B, W, alpha=0.75, beta=1.5)
    assert oracle.relerr(to_np(Ad.grad), dA) <= tol
    assert oracle.relerr(to_np(Bd.grad), dB) <= tol
    assert np.array_equal(to_np(Cd.grad), dC0)
    # forward value too
    ref = oracle.contract(SPEC, A, B, C0, alpha=0.75, beta=1.5)
    assert oracle.relerr(to_np(C), ref) <= tol


def test_backward_finite_differences_12_extent():
    """Central differences (h = 1e-6) of the GPU FP64 forward over every one
    of the 2 x 20736 entries of A and B of the 12-extent copy.

    The perturbed forwards are evaluated together: stacking T perturbed
    copies of A along a new free label t turns them into one contraction
    "tabij=tacik*bkcj" whose slice t is the forward at A + h e_t, and the loss
    of every slice is the contraction "t=tabij*abij" with W.  Both run through
    the library; the loss is bilinear, so the differences carry rounding
    error only (about eps * |L| / h)."""
    ext, A, B, C0, W = ccsd_inputs(12, 12, 910)
    print_case("fd 12 (all entries)")
    Ad = torch_dev(A, torch.float64)
    Bd = torch_dev(B, torch.float64)
    Wd = torch_dev(W, torch.float64)
    Ag = Ad.clone().requires_grad_(True)
    Bg = Bd.clone().requires_grad_(True)
    (comet.contract_ad(SPEC, Ag, Bg) * Wd).sum().backward()
    h = 1e-6
    c, a, b = oracle.split_spec(SPEC)
    for X, other, grad, which in ((Ad, Bd, Ag.grad, "A"), (Bd, Ad, Bg.grad, "B")):
        n = X.numel()
        stacked = "t%s=t%s*%s" % (c, a, b) if which == "A" else "t%s=%s*t%s" % (c, a, b)
        fd = torch.empty(n, dtype=torch.float64, device=X.device)
        chunk = 5184
        for t0 in range(0, n, chunk):
            T = min(chunk, n - t0)
            idx = torch.arange(T, device=X.device)
            L = []
            for sign in (1.0, -1.0):
                Xt = X.reshape(1, -1).repeat(T, 1)
                Xt[idx, t0 + idx] += sign * h
                Xt = Xt.view((T,) + tuple(X.shape))
                Ct = comet.contract(stacked, Xt, other) if which == "A" else comet.contract(stacked, other, Xt)
                L.append(comet.contract("t=t%s*%s" % (c, c), Ct, Wd))
            fd[t0:t0 + T] = (L[0] - L[1]) / (2 * h)
        got = to_np(grad).reshape(-1)
        assert oracle.relerr(got, to_np(fd)) <= 1e-6, which


def test_adjoint_identity_on_gpu():
    ext, A, B, C0, W = ccsd_inputs(40, 12, 920)
    print_case("adjoint")
    X = torch_dev(A, torch.float64)
    Bd = torch_dev(B, torch.float64)
    Y = torch_dev(W, torch.float64)
    sa, sb = oracle.grad_specs(SPEC)
    lhs = float((Y * comet.contract(SPEC, X, Bd)).sum())
    rhs = float((comet.contract(sa, Y, Bd) * X).sum())
    rhs2 = float((comet.contract(sb, X, Y) * Bd).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert abs(lhs - rhs2) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("spec", ["abcijk=daij*bcdk", "ajbi=kcia*cjkb", "abcd=aebf*dfce"])
def test_backward_other_patterns(spec):
    c, a, b = oracle.split_spec(spec)
    rng = np.random.default_rng(7)
    ext = {ch: int(rng.integers(3, 9)) for ch in set(a + b)}
    A = synth.uniform(930, shape_of(a, ext))
    B = synth.uniform(931, shape_of(b, ext))
    W = synth.uniform(932, shape_of(c, ext))
    print_case("backward", spec)
    Ad = torch_dev(A, torch.float64).requires_grad_(True)
    Bd = torch_dev(B, torch.float64).requires_grad_(True)
    (comet.contract_ad(spec, Ad, Bd, alpha=-2.0) * torch_dev(W, torch.float64)).sum().backward()
    dA, dB, _ = oracle.grad(spec, A, B, W, alpha=-2.0)
    assert oracle.relerr(to_np(Ad.grad), dA) <= 1e-12
    assert oracle.relerr(to_np(Bd.grad), dB) <= 1e-12


def test_backward_fp32_storage():
    ext, A, B, C0, W = ccsd_inputs(24, 8, 940)
    A32, B32, W32 = A.astype(np.float32), B.astype(np.float32), W.astype(np.float32)
    print_case("backward f32")
    Ad = torch_dev(A32, torch.float32).requires_grad_(True)
    Bd = torch_dev(B32, torch.float32).requires_grad_(True)
    (comet.contract_ad(SPEC, Ad, Bd) * torch_dev(W32, torch.float32)).sum().backward()
    dA, dB, _ = oracle.grad(SPEC, A32, B32, W32)
    assert oracle.relerr(to_np(Ad.grad), dA) <= 1e-5
    assert oracle.relerr(to_np(Bd.grad), dB) <= 1e-5
