"""The persistent batched launch and HIP-graph capture.

Each problem of a batch is checked against the oracle (FP64 <= 1e-12, FP32 and
BF16x3 <= 1e-5, integer inputs bit for bit) and against the single-call path;
graph replays are checked against eager results, with eager work and
synchronizations between the replays.
"""
import numpy as np
import pytest

from gpu_common import oracle, print_case, shape_of, synth, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

TDT = {"f64": torch.float64, "f32": torch.float32}
NPT = {"f64": np.float64, "f32": np.float32}


def make_batch(n, seed, dtype, extents=(8, 16, 24, 32), kind="uniform", beta=0.0):
    probs = synth.batch_problems(n, seed, extents)
    out = []
    for i, (spec, ext) in enumerate(probs):
        c, a, b = oracle.split_spec(spec)
        gen = synth.integers if kind == "integer" else synth.uniform
        A = gen(seed * 1000 + 10 * i + 1, shape_of(a, ext)).astype(NPT[dtype])
        B = gen(seed * 1000 + 10 * i + 2, shape_of(b, ext)).astype(NPT[dtype])
        C0 = gen(seed * 1000 + 10 * i + 3, shape_of(c, ext)).astype(NPT[dtype])
        out.append(dict(spec=spec, A=A, B=B, C0=C0, alpha=1.0 if i % 3 else -0.5, beta=beta))
    return out


def to_device(batch, dtype):
    dev = []
    for p in batch:
        dev.append(dict(spec=p["spec"], A=torch_dev(p["A"], TDT[dtype]), B=torch_dev(p["B"], TDT[dtype]),
                        C=torch_dev(p["C0"], TDT[dtype]), alpha=p["alpha"], beta=p["beta"]))
    return dev


@pytest.mark.parametrize("dtype,compute,tol", [("f64", "default", 1e-12), ("f32", "default", 1e-5),
                                               ("f32", "split_bf16x3", 1e-5)])
def test_batch_matches_oracle(dtype, compute, tol):
    host = make_batch(40, 3, dtype, beta=1.0)
    dev = to_device(host, dtype)
    print_case("batch", dtype, compute)
    b = comet.Batch(dev, dtype=TDT[dtype], compute=compute)
    b()
    torch.cuda.synchronize()
    for p, d in zip(host, dev):
        ref = oracle.contract(p["spec"], p["A"], p["B"], p["C0"], alpha=p["alpha"], beta=p["beta"])
        assert oracle.relerr(to_np(d["C"]), ref) <= tol, p["spec"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_integer_bitwise_and_equal_to_single_calls(dtype, monkeypatch):
    host = make_batch(24, 4, dtype, kind="integer", beta=1.0)
    dev = to_device(host, dtype)
    print_case("batch int", dtype)
    comet.Batch(dev, dtype=TDT[dtype])()
    torch.cuda.synchronize()
    monkeypatch.setenv("COMET_GETT_TILE", "1")   # the batch's 64 x 64 tile
    for p, d in zip(host, dev):
        ref = oracle.contract(p["spec"], p["A"], p["B"], p["C0"], alpha=p["alpha"], beta=p["beta"])
        assert np.array_equal(to_np(d["C"]), ref), p["spec"]
        single = comet.contract(p["spec"], torch_dev(p["A"], TDT[dtype]), torch_dev(p["B"], TDT[dtype]),
                                torch_dev(p["C0"], TDT[dtype]), alpha=p["alpha"], beta=p["beta"])
        torch.cuda.synchronize()
        assert torch.equal(single, d["C"])


def test_batch_fused_bf16x3_equals_single_call():
    host = make_batch(16, 5, "f32", beta=0.0)
    dev = to_device(host, "f32")
    print_case("batch bf16x3 vs single")
    comet.Batch(dev, dtype=torch.float32, compute="split_bf16x3")()
    torch.cuda.synchronize()
    for p, d in zip(host, dev):
        single = comet.contract(p["spec"], torch_dev(p["A"], torch.float32), torch_dev(p["B"], torch.float32),
                                alpha=p["alpha"], compute="split_bf16x3")
        torch.cuda.synchronize()
        assert torch.equal(single, d["C"])


def test_batch_degenerate_problems():
    """Empty summation, alpha = 0 and empty outputs inside one batch."""
    print_case("batch degenerate")
    f = torch.float64
    A0 = torch.zeros((6, 0), dtype=f, device="cuda")
    B0 = torch.zeros((0, 5), dtype=f, device="cuda")
    C0 = torch_dev(synth.uniform(1, (6, 5)), f)
    C0ref = C0.clone()
    A1 = torch_dev(synth.uniform(2, (4, 3)), f)
    B1 = torch_dev(synth.uniform(3, (3, 7)), f)
    C1 = torch_dev(synth.uniform(4, (4, 7)), f)
    C1ref = C1.clone()
    A2 = torch.zeros((0, 3), dtype=f, device="cuda")
    B2 = torch_dev(synth.uniform(5, (3, 2)), f)
    C2 = torch.zeros((0, 2), dtype=f, device="cuda")
    A3 = torch_dev(synth.uniform(6, (9, 11)), f)
    B3 = torch_dev(synth.uniform(7, (11, 13)), f)
    C3 = torch.zeros((9, 13), dtype=f, device="cuda")
    probs = [dict(spec="ij=ik*kj", A=A0, B=B0, C=C0, beta=2.0),
             dict(spec="ij=ik*kj", A=A1, B=B1, C=C1, alpha=0.0, beta=-1.0),
             dict(spec="ij=ik*kj", A=A2, B=B2, C=C2),
             dict(spec="ij=ik*kj", A=A3, B=B3, C=C3)]
    comet.Batch(probs, dtype=f)()
    torch.cuda.synchronize()
    assert torch.equal(C0, 2.0 * C0ref)
    assert torch.equal(C1, -1.0 * C1ref)
    ref = oracle.contract("ij=ik*kj", to_np(A3), to_np(B3))
    assert oracle.relerr(to_np(C3), ref) <= 1e-12


def test_batch_forward_and_backward_in_one_launch():
    """loss = sum(C * W): dA and dB do not need C, so the forward problems and
    both gradient contractions of every problem run in one launch."""
    n = 12
    host = make_batch(n, 6, "f64", beta=0.0)
    f = torch.float64
    probs, grads = [], []
    for i, p in enumerate(host):
        c, a, b = oracle.split_spec(p["spec"])
        W = synth.uniform(9000 + i, p["C0"].shape)
        Ad, Bd, Wd = torch_dev(p["A"], f), torch_dev(p["B"], f), torch_dev(W, f)
        C = torch.empty(p["C0"].shape, dtype=f, device="cuda")
        dA = torch.empty(p["A"].shape, dtype=f, device="cuda")
        dB = torch.empty(p["B"].shape, dtype=f, device="cuda")
        sa, sb = oracle.grad_specs(p["spec"])
        probs += [dict(spec=p["spec"], A=Ad, B=Bd, C=C, alpha=p["alpha"]),
                  dict(spec=sa, A=Wd, B=Bd, C=dA, alpha=p["alpha"]),
                  dict(spec=sb, A=Ad, B=Wd, C=dB, alpha=p["alpha"])]
        grads.append((p, W, C, dA, dB))
    print_case("batch fwd+bwd")
    comet.Batch(probs, dtype=f)()
    torch.cuda.synchronize()
    for p, W, C, dA, dB in grads:
        ref = oracle.contract(p["spec"], p["A"], p["B"], alpha=p["alpha"])
        gA, gB, _ = oracle.grad(p["spec"], p["A"], p["B"], W, alpha=p["alpha"])
        assert oracle.relerr(to_np(C), ref) <= 1e-12
        assert oracle.relerr(to_np(dA), gA) <= 1e-12
        assert oracle.relerr(to_np(dB), gB) <= 1e-12


@pytest.mark.parametrize("compute", ["default", "split_bf16x3"])
def test_batch_graph_capture_and_replay(compute):
    host = make_batch(20, 7, "f32", beta=0.0)
    dev = to_device(host, "f32")
    b = comet.Batch(dev, dtype=torch.float32, compute=compute)
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    print_case("batch graph", compute)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b(workspace=ws)          # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b(workspace=ws)
    torch.cuda.synchronize()
    for rep in range(4):
        # change the inputs in place between replays, with eager work around
        for i, (p, d) in enumerate(zip(host, dev)):
            newA = synth.uniform(777 + 31 * rep + i, p["A"].shape).astype(np.float32)
            d["A"].copy_(torch.from_numpy(newA))
            p["A"] = newA
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eager = [d["C"].clone() for d in dev]
        b(workspace=ws)
        torch.cuda.synchronize()
        for d, e in zip(dev, eager):
            assert torch.equal(d["C"], e)
        p0 = host[rep]
        ref = oracle.contract(p0["spec"], p0["A"], p0["B"], alpha=p0["alpha"])
        assert oracle.relerr(to_np(eager[rep]), ref) <= 1e-5


@pytest.mark.parametrize("compute,path,sk", [("f64", "gett", None), ("f64", "ttgt", None), ("split_bf16", "auto", None),
                                             ("split_fp16x2", "auto", None), ("f64", "gett", "16,40"),
                                             ("f64", "ttgt", "5,9")])
def test_plan_graph_capture_and_replay(compute, path, sk, monkeypatch):
    if sk:
        # a stream-K schedule: partial tiles in the workspace, a fixup launch
        monkeypatch.setenv("COMET_GETT_TILE", "3")
        monkeypatch.setenv("COMET_GETT_SK", sk)
    spec = "abij=acik*bkcj"
    # j even: 16-byte vector loads of B, which the stream-K kernels require
    ext = dict(a=20, b=18, c=22, i=9, j=8 if sk else 7, k=10)
    A = synth.uniform(1, shape_of("acik", ext))
    B = synth.uniform(2, shape_of("bkcj", ext))
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    C = torch.zeros(shape_of("abij", ext), dtype=torch.float64, device="cuda")
    plan = comet.Plan(spec, Ad, Bd, C, compute=compute, path=path)
    ws = plan.workspace(Ad.device)
    print_case("plan graph", compute, path, sk)
    if sk:
        assert plan.workspace_bytes > 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan(Ad, Bd, C)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan(Ad, Bd, C, workspace=ws)
    torch.cuda.synchronize()
    tol = 1e-12 if compute == "f64" else (1e-9 if compute == "split_bf16" else 1e-5)
    for rep in range(4):
        A = synth.uniform(100 + rep, A.shape)
        Ad.copy_(torch.from_numpy(A))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = to_np(C)
        assert oracle.relerr(got, oracle.contract(spec, A, B)) <= tol
        C2 = plan(Ad, Bd)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(C2), got)


def test_contract_refuses_capture():
    """The convenience call owns a workspace it may need to grow: it refuses
    to run under capture (the plan API is the capturable one)."""
    A = torch.ones((4, 5), dtype=torch.float64, device="cuda")
    B = torch.ones((5, 6), dtype=torch.float64, device="cuda")
    comet.contract("ij=ik*kj", A, B)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g):
        try:
            comet.contract("ij=ik*kj", A, B)
        except comet.CometError as e:
            err = e
    assert err is not None and err.name == "UNSUPPORTED"


@pytest.mark.parametrize("cls", [0, 1, 2, 3])
@pytest.mark.parametrize("kind", ["integer", "uniform"])
def test_batch_each_tile_class_matches_oracle(cls, kind, monkeypatch):
    """Every tile class of the FP32 batch forced through COMET_BATCH_CLASS on
    problems with ragged extents (not multiples of the class tile): bit-exact
    on integer inputs, <= 1e-5 otherwise; element-load problems keep class 0."""
    host = make_batch(30, 20 + cls, "f32", extents=(8, 16, 24, 40, 56, 72), kind=kind, beta=1.0)
    dev = to_device(host, "f32")
    monkeypatch.setenv("COMET_BATCH_CLASS", str(cls))
    print_case("batch class", cls, kind)
    b = comet.Batch(dev, dtype=torch.float32)
    d = b.describe()
    assert d["classes"][cls] > 0 and sum(d["classes"]) == len(host)
    b()
    torch.cuda.synchronize()
    for p, x in zip(host, dev):
        ref = oracle.contract(p["spec"], p["A"], p["B"], p["C0"], alpha=p["alpha"], beta=p["beta"])
        if kind == "integer":
            assert np.array_equal(to_np(x["C"]), ref), p["spec"]
        else:
            assert oracle.relerr(to_np(x["C"]), ref) <= 1e-5, p["spec"]


def test_batch_model_and_queues_describe():
    """The untuned class choice and the queues: every problem is in exactly
    one class, the queues hold every output tile, and each queue is used."""
    host = make_batch(64, 31, "f32", extents=(8, 32, 64))
    dev = to_device(host, "f32")
    print_case("batch describe")
    d = comet.Batch(dev, dtype=torch.float32).describe()
    assert sum(d["classes"]) == 64 and d["tuned"] == 0
    assert sum(d["queues"]) == d["tiles"] and min(d["queues"]) > 0


@pytest.mark.parametrize("copy", ["1", "0"])
def test_batch_element_load_problems_copy_or_gather(copy, monkeypatch):
    """Problems of the patterns whose operands have their unit strides on
    different summation labels: by default one operand is copied into a
    vector-readable order before the launch, COMET_BATCH_COPY=0 gathers them
    element by element; both bit-exact on integer inputs, twice in a row
    with new input values in between (the copy is refreshed every execute)."""
    specs = ["abij=ciak*bkjc", "cjkb=kcia*ajbi", "abij=acik*bkcj"]
    monkeypatch.setenv("COMET_BATCH_COPY", copy)
    rng = np.random.default_rng(5)
    host = []
    for t in range(12):
        spec = specs[t % 3]
        c, a, b = oracle.split_spec(spec)
        ext = {ch: int(rng.choice([8, 16, 24, 40])) for ch in set(a + b)}
        A = synth.integers(900 + 10 * t, shape_of(a, ext)).astype(np.float32)
        B = synth.integers(901 + 10 * t, shape_of(b, ext)).astype(np.float32)
        host.append(dict(spec=spec, A=A, B=B, C0=np.zeros(shape_of(c, ext), np.float32), alpha=1.0, beta=0.0))
    dev = to_device(host, "f32")
    print_case("batch copies", copy)
    bt = comet.Batch(dev, dtype=torch.float32)
    d = bt.describe()
    assert (d["copies"] > 0) == (copy == "1")
    for rep in range(2):
        if rep == 1:
            for p, x in zip(host, dev):
                p["A"] = -2.0 * p["A"] + 1.0
                x["A"].copy_(torch_dev(p["A"], torch.float32))
        bt()
        torch.cuda.synchronize()
        for p, x in zip(host, dev):
            assert np.array_equal(to_np(x["C"]), oracle.contract(p["spec"], p["A"], p["B"])), (rep, p["spec"])
