"""The batched workload at its real size: 1024 problems of the six patterns,
every label's extent from {8, ..., 64}, forward + dA + dB (3072
contractions) in one persistent launch captured in a HIP graph, in FP32 and
in BF16x3.

* uniform[-1, 1] inputs: every contraction of every problem is checked
  against the oracle at 64 output points (both corners included), relative
  error <= 1e-5 (the FP32-class bound; BF16x3 on FP32 storage is held to it
  too, since rounding the output to FP32 alone exceeds 1e-9);
* integer inputs in [-3, 3] (every product and partial sum is an integer
  below 2^24, exact in FP32 and in the BF16 slices): the seeded sample of
  synth.batch_check_sample (128 problems, every problem of at most 2^24
  FLOPs and the 20 heaviest) is compared with the oracle bit for bit, at the
  points and, for problems of at most 2^26 FLOPs, over the whole output;
* graph replays give the bits of the eager launch."""
import numpy as np
import pytest

from gpu_common import oracle, print_case, shape_of, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

N_PROBLEMS = 1024
POINTS = 64


def _labels(spec):
    c, a, b = oracle.split_spec(spec)
    return c, a, b


def _workload(kind):
    dev = torch.device("cuda:0")
    gen = synth.uniform_torch if kind == "uniform" else synth.integers_torch
    probs = synth.batch_problems(N_PROBLEMS, synth.config_seed(5, "A"))
    tensors, problems = [], []
    for i, (spec, ext) in enumerate(probs):
        c, a, b = _labels(spec)
        A = gen(5_100_000 + 10 * i + 1, shape_of(a, ext), torch.float32, dev)
        B = gen(5_100_000 + 10 * i + 2, shape_of(b, ext), torch.float32, dev)
        W = gen(5_100_000 + 10 * i + 4, shape_of(c, ext), torch.float32, dev)
        C = torch.full(shape_of(c, ext), float("nan"), dtype=torch.float32, device=dev)
        dA, dB = torch.full_like(A, float("nan")), torch.full_like(B, float("nan"))
        sa, sb = oracle.grad_specs(spec)
        problems += [dict(spec=spec, A=A, B=B, C=C), dict(spec=sa, A=W, B=B, C=dA), dict(spec=sb, A=A, B=W, C=dB)]
        tensors.append((spec, ext, A, B, W, C, dA, dB))
    return probs, tensors, problems


def _points(shape, seed):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, e, POINTS - 2) for e in shape], axis=1).reshape(POINTS - 2, len(shape))
    return np.concatenate([np.zeros((1, len(shape)), np.int64), np.array([shape], np.int64) - 1, pts])


def _run(problems, mode, snap_ids, tensors):
    batch = comet.Batch(problems, dtype=torch.float32, compute=mode)
    ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch(workspace=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    eager = {i: [t.clone() for t in tensors[i][5:]] for i in snap_ids}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch(workspace=ws)
    for _ in range(2):
        for i in snap_ids:
            for t in tensors[i][5:]:
                t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for i in snap_ids:
            for x, y in zip(eager[i], tensors[i][5:]):
                assert torch.equal(x, y), "graph replay differs from the eager launch (problem %d)" % i
    del g, batch


def _check_points(i, spec, ext, A, B, W, C, dA, dB, tol):
    """(max relative error over the three contractions, exact?) at POINTS points each."""
    c, a, b = _labels(spec)
    sa, sb = oracle.grad_specs(spec)
    An, Bn, Wn = (x.double().cpu().numpy() for x in (A, B, W))
    worst, exact = 0.0, True
    for sp, X, Y, got, lab in ((spec, An, Bn, C, c), (sa, Wn, Bn, dA, a), (sb, An, Wn, dB, b)):
        pts = _points(shape_of(lab, ext), 1000 + i)
        ref = oracle.contract_points(sp, X, Y, pts)
        g = got.double().cpu().numpy()[tuple(pts.T)]
        assert np.all(np.isfinite(g)), "problem %d %s: unwritten outputs" % (i, sp)
        worst = max(worst, oracle.relerr(g, ref))
        exact = exact and np.array_equal(g, ref)
    return worst, exact


@pytest.mark.parametrize("mode", ["default", "split_bf16x3"])
def test_batch_full_size_uniform(mode):
    print_case("batch full uniform", mode)
    probs, tensors, problems = _workload("uniform")
    _run(problems, mode, [0, 1, N_PROBLEMS - 1], tensors)
    worst = 0.0
    for i, (spec, ext, A, B, W, C, dA, dB) in enumerate(tensors):
        err, _ = _check_points(i, spec, ext, A, B, W, C, dA, dB, 1e-5)
        assert err <= 1e-5, "problem %d (%s %s): relerr %.3e" % (i, spec, ext, err)
        worst = max(worst, err)
        if i % 128 == 127:
            print("[progress] %s checked %d problems, worst %.2e" % (mode, i + 1, worst), flush=True)
    del tensors, problems
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["default", "split_bf16x3"])
def test_batch_full_size_integer_exact(mode):
    print_case("batch full integer", mode)
    probs, tensors, problems = _workload("integer")
    sample = synth.batch_check_sample(probs)
    assert len(sample) >= 128
    flops = [2.0 * np.prod(list(ext.values())) for _, ext in probs]
    top20 = sorted(flops)[-20]
    assert sum(1 for i in sample if flops[i] >= top20) >= 20   # the 20 heaviest (ties either way)
    _run(problems, mode, sample[:4], tensors)
    for n, i in enumerate(sample):
        spec, ext, A, B, W, C, dA, dB = tensors[i]
        _, exact = _check_points(i, spec, ext, A, B, W, C, dA, dB, 0.0)
        assert exact, "problem %d (%s %s) not bit-exact" % (i, spec, ext)
        if 2.0 * np.prod(list(ext.values())) <= 2.0 ** 26:
            An, Bn, Wn = (x.double().cpu().numpy() for x in (A, B, W))
            sa, sb = oracle.grad_specs(spec)
            assert np.array_equal(C.double().cpu().numpy(), oracle.contract(spec, An, Bn))
            assert np.array_equal(dA.double().cpu().numpy(), oracle.contract(sa, Wn, Bn))
            assert np.array_equal(dB.double().cpu().numpy(), oracle.contract(sb, An, Wn))
        if n % 32 == 31:
            print("[progress] %s checked %d of %d sampled problems" % (mode, n + 1, len(sample)), flush=True)
    del tensors, problems
    torch.cuda.empty_cache()
