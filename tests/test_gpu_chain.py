"""Multi-operand chains on the GPU (comet_contract_chain): the result of the
chosen grouping against the oracle applied pairwise in the natural order (the
chain reassociation pin), bit for bit on integer inputs."""
import numpy as np
import pytest

from gpu_common import oracle, print_case, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")


def parse(spec):
    out, rhs = spec.replace(" ", "").split("=")
    return out, rhs.split("*")


def oracle_chain(spec, arrays, alpha=1.0, beta=0.0, C0=None):
    """Left to right with the oracle: T = A1*A2, T = T*A3, ..., keeping the
    labels still needed."""
    out, ops = parse(spec)
    acc, lab = arrays[0], ops[0]
    for i in range(1, len(ops)):
        rest = set(out).union(*[set(o) for o in ops[i + 1:]])
        keep = "".join(l for l in dict.fromkeys(lab + ops[i]) if l in rest)
        if i == len(ops) - 1:
            keep = out
        acc = oracle.contract("%s=%s*%s" % (keep, lab, ops[i]), acc, arrays[i],
                              C0 if i == len(ops) - 1 else None,
                              alpha=alpha if i == len(ops) - 1 else 1.0, beta=beta if i == len(ops) - 1 else 0.0)
        lab = keep
    return acc


CASES = [
    ("abil=acik*cbkj*jl", dict(a=9, b=7, i=6, l=5, c=8, k=4, j=6)),
    ("ai=cdmn*inad*mc", dict(a=12, i=10, c=3, d=11, m=9, n=7)),
    ("ij=ik*kl*lm*mj", dict(i=40, k=5, l=33, m=6, j=29)),
    ("abij=mnef*am*fn*ebij", dict(a=10, b=9, i=5, j=6, m=4, n=5, e=11, f=7)),
    # labels in more than two tensors
    ("bij=bik*bkl*blj", dict(b=5, i=30, k=4, l=50, j=3)),
    ("aij=aik*kl*alj*ij", dict(a=7, i=9, k=11, l=13, j=5)),
]


@pytest.mark.parametrize("spec,ext", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_chain_matches_oracle(spec, ext, dtype):
    out, ops = parse(spec)
    print_case("chain", spec, dtype)
    ints = [synth.integers(40 + i, tuple(ext[l] for l in o)) for i, o in enumerate(ops)]
    got = comet.contract_chain(spec, [torch_dev(x, dtype) for x in ints])
    torch.cuda.synchronize()
    assert np.array_equal(to_np(got), oracle_chain(spec, ints))
    vals = [synth.uniform(50 + i, tuple(ext[l] for l in o)) for i, o in enumerate(ops)]
    cast = np.float64 if dtype == torch.float64 else np.float32
    vals = [v.astype(cast) for v in vals]
    C0 = synth.uniform(60, tuple(ext[l] for l in out)).astype(cast)
    Cd = torch_dev(C0, dtype)
    comet.contract_chain(spec, [torch_dev(x, dtype) for x in vals], Cd, alpha=0.5, beta=-2.0)
    torch.cuda.synchronize()
    ref = oracle_chain(spec, vals, alpha=0.5, beta=-2.0, C0=C0)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert oracle.relerr(to_np(Cd), ref) <= tol


def test_chain_strided_operand_and_capture_refusal():
    spec, ext = CASES[0]
    out, ops = parse(spec)
    arrs = [synth.uniform(70 + i, tuple(ext[l] for l in o)) for i, o in enumerate(ops)]
    big = torch_dev(synth.uniform(80, (ext["j"], 3 * ext["l"])), torch.float64)
    view = big[:, ::3]                                      # jl operand as a strided view
    arrs[2] = to_np(view).copy()
    got = comet.contract_chain(spec, [torch_dev(arrs[0], torch.float64), torch_dev(arrs[1], torch.float64), view])
    torch.cuda.synchronize()
    assert oracle.relerr(to_np(got), oracle_chain(spec, arrs)) <= 1e-12
    g = torch.cuda.CUDAGraph()
    err = None
    ts = [torch_dev(a, torch.float64) for a in arrs]
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        try:
            comet.contract_chain(spec, ts)
        except comet.CometError as e:
            err = e
    assert err is not None and err.name == "UNSUPPORTED"
