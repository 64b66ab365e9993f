"""Every TTGT flattening (Section 6, "Optimal permutation for TTGT": each
order of the M, N and K label groups, each operand stored K-major or not,
with and without exchanging A and B) forced through COMET_TTGT_ORDER on two
small problems, each compared with the oracle bit for bit on integer inputs
with beta != 0."""
import itertools

import numpy as np
import pytest

from gpu_common import oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")


def flattenings(spec):
    c, a, b = oracle.split_spec(spec)
    M = [l for l in a if l in c]
    N = [l for l in b if l in c]
    K = [l for l in a if l not in c]
    rows = set()
    for mo in itertools.permutations(M):
        for no in itertools.permutations(N):
            for ko in itertools.permutations(K):
                mo_, no_, ko_ = "".join(mo), "".join(no), "".join(ko)
                for swap, la, lb in itertools.product((0, 1), repeat=3):
                    r_, c_ = (no_, mo_) if swap else (mo_, no_)
                    left = ko_ + r_ if la else r_ + ko_
                    right = c_ + ko_ if lb else ko_ + c_
                    ap, bp = (right, left) if swap else (left, right)
                    rows.add((ap, bp, r_ + c_))
    return sorted(rows)


CASES = [
    ("abij=acik*bkcj", dict(a=6, b=5, c=7, i=3, j=4, k=5), 64),
    ("abcijk=daij*bcdk", dict(a=4, b=3, c=5, d=6, i=2, j=3, k=4), 288),
]


@pytest.mark.parametrize("spec,ext,count", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_every_ttgt_flattening_is_exact(spec, ext, count, dtype, monkeypatch):
    c, a, b = oracle.split_spec(spec)
    A = synth.integers(8301, shape_of(a, ext))
    B = synth.integers(8302, shape_of(b, ext))
    C0 = synth.integers(8303, shape_of(c, ext))
    ref = oracle.contract(spec, A, B, C0, alpha=2.0, beta=-1.0)
    Ad, Bd, C0d = torch_dev(A, dtype), torch_dev(B, dtype), torch_dev(C0, dtype)
    rows = flattenings(spec)
    assert len(rows) == count
    print_case("ttgt flattenings", spec, dtype, len(rows))
    for ap, bp, cp in rows:
        monkeypatch.setenv("COMET_TTGT_ORDER", "%s|%s|%s" % (ap, bp, cp))
        plan = comet.Plan(spec, Ad, Bd, C0d, path="ttgt")
        t = plan.describe()["ttgt"]
        assert (t["A"], t["B"], t["C"]) == (ap, bp, cp)
        C = C0d.clone()
        plan(Ad, Bd, C, alpha=2.0, beta=-1.0)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(C), ref), (ap, bp, cp)
        del plan
    monkeypatch.delenv("COMET_TTGT_ORDER")
