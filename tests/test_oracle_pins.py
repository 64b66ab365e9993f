"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each check is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign, a wrong stride or label, a transposed operand, a mishandled
alpha/beta) fails at least one of them; tests/test_oracle_mutants.py plants
such slips in a copy of the oracle and confirms it.
"""
import itertools
import os
import random

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_spec(rng, max_per_class=3, allow_empty_k=True):
    """A random valid binary-contraction spec: M labels (A and C), N (B and C), K (A and B)."""
    letters = list("abcdefghijklmnopqrstuvwxyzABCDEFGHIJ")
    rng.shuffle(letters)
    nm = rng.randint(0, max_per_class)
    nn = rng.randint(0, max_per_class)
    nk = rng.randint(0 if allow_empty_k else 1, max_per_class)
    m = letters[:nm]
    n = letters[nm:nm + nn]
    k = letters[nm + nn:nm + nn + nk]
    a = m + k
    b = k + n
    c = m + n
    rng.shuffle(a)
    rng.shuffle(b)
    rng.shuffle(c)
    return "%s=%s*%s" % ("".join(c), "".join(a), "".join(b))


def random_extents(rng, spec, lo=1, hi=4):
    return {ch: rng.randint(lo, hi) for ch in set(spec) if ch.isalpha()}


def shape_of(labels, ext):
    return tuple(ext[ch] for ch in labels)


def make_inputs(spec, ext, seed, integer=False, beta=False):
    c, a, b = oracle.split_spec(spec)
    gen = synth.integers if integer else synth.uniform
    A = gen(seed + 1, shape_of(a, ext))
    B = gen(seed + 2, shape_of(b, ext))
    C0 = gen(seed + 3, shape_of(c, ext)) if beta else None
    return A, B, C0


def einsum(spec, A, B):
    c, a, b = oracle.split_spec(spec)
    return np.einsum("%s,%s->%s" % (a, b, c), A, B)


def python_loop(spec, A, B, C0, alpha, beta):
    """The definition written out with Python loops (tiny inputs only)."""
    c, a, b = oracle.split_spec(spec)
    ext = {}
    for labs, arr in ((a, A), (b, B)):
        for ch, n in zip(labs, arr.shape):
            ext[ch] = n
    ksum = [ch for ch in a if ch not in c]
    out = np.zeros(tuple(ext[ch] for ch in c))
    for cidx in itertools.product(*[range(ext[ch]) for ch in c]):
        val = dict(zip(c, cidx))
        s = 0.0
        if alpha != 0.0:
            for kidx in itertools.product(*[range(ext[ch]) for ch in ksum]):
                val.update(zip(ksum, kidx))
                s = s + float(A[tuple(val[ch] for ch in a)]) * float(B[tuple(val[ch] for ch in b)])
        r = alpha * s
        if beta != 0.0:
            r = r + beta * float(C0[cidx])
        out[cidx] = r
    return out


# --------------------------------------------------------------------------
# brute force, Python loops, einsum
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", range(60))
def test_oracle_equals_python_loop_bitwise(case):
    rng = random.Random(1000 + case)
    spec = random_spec(rng, max_per_class=2)
    ext = random_extents(rng, spec, 1, 3)
    A, B, C0 = make_inputs(spec, ext, 7000 + 10 * case, beta=True)
    alpha, beta = 0.75, (0.0 if case % 3 == 0 else -1.25)
    got = oracle.contract(spec, A, B, C0, alpha=alpha, beta=beta)
    ref = python_loop(spec, A, B, C0, alpha, beta)
    assert np.array_equal(got, ref), spec


@pytest.mark.parametrize("case", range(80))
def test_oracle_equals_bruteforce(case):
    rng = random.Random(2000 + case)
    spec = random_spec(rng)
    ext = random_extents(rng, spec)
    integer = case % 2 == 1
    A, B, C0 = make_inputs(spec, ext, 9000 + 10 * case, integer=integer, beta=True)
    beta = 0.0 if case % 4 == 0 else 2.0
    got = oracle.contract(spec, A, B, C0, alpha=-1.5, beta=beta)
    ref = oracle.bruteforce(spec, A, B, C0, alpha=-1.5, beta=beta)
    if integer:
        assert np.array_equal(got, ref), spec
    else:
        assert oracle.relerr(got, ref) <= 1e-14, spec
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("case", range(80))
def test_oracle_equals_einsum(case):
    rng = random.Random(3000 + case)
    spec = random_spec(rng)
    ext = random_extents(rng, spec, 1, 5)
    A, B, _ = make_inputs(spec, ext, 11000 + 10 * case)
    got = oracle.contract(spec, A, B)
    ref = einsum(spec, A, B)
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-14), spec


@pytest.mark.parametrize("case", range(40))
def test_oracle_integer_inputs_exact_vs_integer_einsum(case):
    """Integer-valued inputs: every partial sum is an exact integer in FP64,
    so the oracle must equal numpy's exact int64 einsum bit for bit."""
    rng = random.Random(4000 + case)
    spec = random_spec(rng)
    ext = random_extents(rng, spec, 1, 5)
    A, B, C0 = make_inputs(spec, ext, 13000 + 10 * case, integer=True, beta=True)
    got = oracle.contract(spec, A, B, C0, alpha=3.0, beta=-2.0)
    ref = 3 * einsum(spec, A.astype(np.int64), B.astype(np.int64)) - 2 * C0.astype(np.int64)
    assert np.array_equal(got, ref.astype(np.float64)), spec


# --------------------------------------------------------------------------
# batch labels (in C, A and B: they index all three and are not summed)
# --------------------------------------------------------------------------

def random_batch_spec(rng, max_per_class=2):
    letters = list("abcdefghijklmnopqrstuvwxyz")
    rng.shuffle(letters)
    nx = rng.randint(1, 2)
    nm, nn, nk = (rng.randint(0, max_per_class) for _ in range(3))
    x = letters[:nx]
    m = letters[nx:nx + nm]
    n = letters[nx + nm:nx + nm + nn]
    k = letters[nx + nm + nn:nx + nm + nn + nk]
    a, b, c = x + m + k, x + k + n, x + m + n
    for t in (a, b, c):
        rng.shuffle(t)
    return "%s=%s*%s" % ("".join(c), "".join(a), "".join(b))


@pytest.mark.parametrize("case", range(30))
def test_batch_labels_equal_python_loop_einsum_and_bruteforce(case):
    rng = random.Random(5000 + case)
    spec = random_batch_spec(rng)
    ext = random_extents(rng, spec, 1, 4)
    A, B, C0 = make_inputs(spec, ext, 15000 + 10 * case, integer=case % 2 == 1, beta=True)
    got = oracle.contract(spec, A, B, C0, alpha=0.5, beta=-1.0)
    assert np.array_equal(got, python_loop(spec, A, B, C0, 0.5, -1.0)), spec
    assert np.allclose(oracle.contract(spec, A, B), einsum(spec, A, B), rtol=1e-13, atol=1e-14), spec
    brute = oracle.bruteforce(spec, A, B, C0, alpha=0.5, beta=-1.0)
    if case % 2:
        assert np.array_equal(got, brute), spec
    else:
        assert oracle.relerr(got, brute) <= 1e-14, spec


def test_hadamard_product_closed_form():
    """All labels batch labels: C = A * B elementwise, exactly."""
    A = synth.uniform(121, (5, 7, 3))
    B = synth.uniform(122, (5, 7, 3))
    assert np.array_equal(oracle.contract("ijk=ijk*ijk", A, B), A * B)
    # a batch of matrix products against numpy matmul
    X = synth.uniform(123, (4, 6, 5))
    Y = synth.uniform(124, (4, 5, 7))
    assert oracle.relerr(oracle.contract("bij=bik*bkj", X, Y), np.matmul(X, Y)) <= 1e-15


# --------------------------------------------------------------------------
# closed forms on the benchmark configurations' specs
# --------------------------------------------------------------------------

CONFIG_SPECS = [
    ("abij=acik*cbkj", dict(a=6, b=5, c=7, i=4, j=3, k=5)),
    ("abij=acik*bkcj", dict(a=6, b=5, c=7, i=4, j=3, k=5)),
    ("abcijk=daij*bcdk", dict(a=3, b=4, c=2, d=6, i=3, j=2, k=4)),
]


@pytest.mark.parametrize("spec,ext", CONFIG_SPECS)
def test_all_ones_gives_product_of_contracted_extents(spec, ext):
    c, a, b = oracle.split_spec(spec)
    A = np.ones(shape_of(a, ext))
    B = np.ones(shape_of(b, ext))
    C0 = synth.integers(5, shape_of(c, ext))
    kprod = int(np.prod([ext[ch] for ch in a if ch not in c]))
    got = oracle.contract(spec, A, B, C0, alpha=2.0, beta=1.0)
    assert np.array_equal(got, 2.0 * kprod + C0)
    got0 = oracle.contract(spec, A, B, alpha=0.5)
    assert np.all(got0 == 0.5 * kprod)


def test_all_ones_full_config1():
    A = np.ones((16,) * 4)
    B = np.ones((16,) * 4)
    assert np.all(oracle.contract("abij=acik*cbkj", A, B) == 256.0)


def test_delta_config1_reproduces_A():
    # B[c,b,k,j] = delta_cb delta_kj  =>  C[a,b,i,j] = A[a,b,i,j]
    n = 5
    A = synth.uniform(21, (n, n, n, n))
    B = np.einsum("cb,kj->cbkj", np.eye(n), np.eye(n))
    assert np.array_equal(oracle.contract("abij=acik*cbkj", A, B), A)


def test_delta_config2_reproduces_A():
    # B[b,k,c,j] = delta_bc delta_kj  =>  C[a,b,i,j] = A[a,b,i,j]
    v, o = 6, 4
    A = synth.uniform(22, (v, v, o, o))
    B = np.einsum("bc,kj->bkcj", np.eye(v), np.eye(o))
    assert np.array_equal(oracle.contract("abij=acik*bkcj", A, B), A)


def test_delta_config3_broadcasts_permuted_A():
    # B[b,c,d,k] = delta_bd  =>  C[a,b,c,i,j,k] = A[b,a,i,j] for every c, k
    v, o = 4, 3
    A = synth.uniform(23, (v, v, o, o))           # A[d,a,i,j]
    B = np.einsum("bd,c,k->bcdk", np.eye(v), np.ones(v), np.ones(o))
    got = oracle.contract("abcijk=daij*bcdk", A, B)
    ref = np.broadcast_to(A.transpose(1, 0, 2, 3)[:, :, None, :, :, None], (v, v, v, o, o, o))
    assert np.array_equal(got, ref)


def test_pure_gemm_special_case_matches_matmul():
    a, b, c, d, i, j = 5, 4, 6, 3, 7, 2
    A = synth.uniform(31, (a, b, c, d))
    B = synth.uniform(32, (c, d, i, j))
    got = oracle.contract("abij=abcd*cdij", A, B)
    ref = (A.reshape(a * b, c * d) @ B.reshape(c * d, i * j)).reshape(a, b, i, j)
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_chain_reassociation():
    """(A*B)*D == A*(B*D): contracting the output with a third tensor equals
    the reassociated chain (the associativity that multi-operand ordering
    relies on, Section 6)."""
    ext = dict(a=4, b=3, c=5, i=2, j=4, k=3, l=5)
    A = synth.uniform(41, shape_of("acik", ext))
    B = synth.uniform(42, shape_of("cbkj", ext))
    D = synth.uniform(43, shape_of("jl", ext))
    C = oracle.contract("abij=acik*cbkj", A, B)
    E1 = oracle.contract("abil=abij*jl", C, D)
    BD = oracle.contract("cbkl=cbkj*jl", B, D)
    E2 = oracle.contract("abil=acik*cbkl", A, BD)
    assert oracle.relerr(E1, E2) < 1e-14


def test_worked_example_eq1_ttgt_fixture():
    """The paper's TTGT decomposition of its worked example, executed with
    numpy transposes and a matmul, equals the oracle."""
    fx = {}
    with open(os.path.join(GOLDEN, "eq1_ttgt.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                key, val = line.split(None, 1)
                fx[key] = val
    spec = fx["spec"]
    c, a, b = oracle.split_spec(spec)
    assert set(fx["summation"]) == set(a) & set(b)
    ext = dict(a=3, b=4, c=5, d=2, e=3, f=4)
    A = synth.uniform(51, shape_of(a, ext))
    B = synth.uniform(52, shape_of(b, ext))
    TA = A.transpose([a.index(ch) for ch in fx["TA"]])
    TB = B.transpose([b.index(ch) for ch in fx["TB"]])
    groups = dict(g.split("=") for g in fx["merge"].split())
    mi = int(np.prod([ext[ch] for ch in groups["i"]]))
    mj = int(np.prod([ext[ch] for ch in groups["j"]]))
    mk = int(np.prod([ext[ch] for ch in groups["k"]]))
    assert fx["TA"] == groups["i"] + groups["j"] and fx["TB"] == groups["j"] + groups["k"]
    Cp = TA.reshape(mi, mj) @ TB.reshape(mj, mk)
    TC = Cp.reshape(shape_of(fx["TC"], ext))
    Cref = TC.transpose([fx["TC"].index(ch) for ch in c])
    got = oracle.contract(spec, A, B)
    assert np.allclose(got, Cref, rtol=1e-14, atol=1e-14)


# --------------------------------------------------------------------------
# storage invariances, strides, alpha/beta, edges
# --------------------------------------------------------------------------

def test_storage_permutation_invariance():
    rng = np.random.default_rng(5)
    ext = dict(a=4, b=3, c=5, i=2, j=4, k=3)
    A = synth.uniform(61, shape_of("acik", ext))
    B = synth.uniform(62, shape_of("cbkj", ext))
    ref = oracle.contract("abij=acik*cbkj", A, B)
    # permuting B's storage (and relabeling) keeps each sum's order: bitwise
    for _ in range(5):
        p = rng.permutation(4)
        lab = "".join("cbkj"[q] for q in p)
        Bp = np.ascontiguousarray(B.transpose(p))
        assert np.array_equal(oracle.contract("abij=acik*" + lab, A, Bp), ref)
    # permuting C's storage permutes the output only: bitwise
    for _ in range(5):
        p = rng.permutation(4)
        lab = "".join("abij"[q] for q in p)
        got = oracle.contract(lab + "=acik*cbkj", A, B)
        assert np.array_equal(got, ref.transpose(p))
    # permuting A's storage reorders each sum: equal to rounding
    for _ in range(5):
        p = rng.permutation(4)
        lab = "".join("acik"[q] for q in p)
        got = oracle.contract("abij=%s*cbkj" % lab, np.ascontiguousarray(A.transpose(p)), B)
        assert oracle.relerr(got, ref) < 1e-15


def test_strided_views_equal_contiguous_copies():
    base_A = synth.uniform(71, (9, 8, 7, 6))
    base_B = synth.uniform(72, (7, 9, 8, 10))
    A = base_A[1:7:2, ::3, 1:, 2:5]           # a, c, i, k  (3, 3, 6, 3)
    B = base_B[1:4:1, 0:9:2, ::2, 2:9:3]      # c, b, k, j  (3, 5, 4, 3)
    A = A[:, :, :, :3]
    B = B[:3, :, :3, :]
    got = oracle.contract("abij=acik*cbkj", A, B[:, :, :, :])
    ref = oracle.contract("abij=acik*cbkj", np.ascontiguousarray(A), np.ascontiguousarray(B))
    assert np.array_equal(got, ref)


def test_beta_zero_does_not_read_C():
    spec = "abij=acik*cbkj"
    A = synth.uniform(81, (3, 4, 2, 3))
    B = synth.uniform(82, (4, 3, 3, 2))
    out = np.full((3, 3, 2, 2), np.nan)
    lib = oracle._load()
    dA, sA = oracle._meta(A)
    dB, sB = oracle._meta(B)
    dC, sC = oracle._meta(out)
    rc = lib.oracle_contract(spec.encode(), 1.0, oracle._ptr(A), oracle._ptr(dA), oracle._ptr(sA),
                             oracle._ptr(B), oracle._ptr(dB), oracle._ptr(sB), 0.0,
                             oracle._ptr(out), oracle._ptr(dC), oracle._ptr(sC), 1)
    assert rc == 0
    assert np.all(np.isfinite(out))
    assert np.array_equal(out, oracle.contract(spec, A, B))


def test_alpha_zero_does_not_read_inputs():
    A = np.full((3, 4, 2, 3), np.nan)
    B = np.full((4, 3, 3, 2), np.inf)
    C0 = synth.uniform(83, (3, 3, 2, 2))
    got = oracle.contract("abij=acik*cbkj", A, B, C0, alpha=0.0, beta=0.5)
    assert np.array_equal(got, 0.5 * C0)


def test_dsl_forms_assign_add_subtract():
    """'=' is beta 0, '+=' is beta 1, '-=' is beta 1 with alpha negated."""
    A = synth.integers(84, (3, 4, 2, 3))
    B = synth.integers(85, (4, 3, 3, 2))
    C0 = synth.integers(86, (3, 3, 2, 2))
    P = einsum("abij=acik*cbkj", A, B)
    assert np.array_equal(oracle.contract("abij=acik*cbkj", A, B, C0, 1.0, 0.0), P)
    assert np.array_equal(oracle.contract("abij=acik*cbkj", A, B, C0, 1.0, 1.0), C0 + P)
    assert np.array_equal(oracle.contract("abij=acik*cbkj", A, B, C0, -1.0, 1.0), C0 - P)


def test_outer_product_no_contracted_labels():
    A = synth.uniform(91, (3, 4))
    B = synth.uniform(92, (5,))
    got = oracle.contract("iaj=ij*a", A, B)
    assert np.array_equal(got, A[:, None, :] * B[None, :, None])


def test_full_contraction_to_scalar():
    A = synth.integers(93, (4, 5))
    B = synth.integers(94, (5, 4))
    got = oracle.contract("=ab*ba", A, B)
    assert got.shape == ()
    assert float(got) == float(np.sum(A * B.T))


def test_zero_contracted_extent_gives_beta_C():
    A = np.zeros((3, 0))
    B = np.zeros((0, 4))
    C0 = synth.uniform(95, (3, 4))
    assert np.array_equal(oracle.contract("ij=ik*kj", A, B, C0, 1.0, 2.0), 2.0 * C0)
    assert np.array_equal(oracle.contract("ij=ik*kj", A, B), np.zeros((3, 4)))


def test_zero_free_extent_gives_empty():
    A = np.zeros((0, 3))
    B = synth.uniform(96, (3, 4))
    assert oracle.contract("ij=ik*kj", A, B).shape == (0, 4)


def test_points_equal_full_result():
    spec = "abij=acik*bkcj"
    ext = dict(a=5, b=4, c=6, i=3, j=5, k=4)
    A = synth.uniform(101, shape_of("acik", ext))
    B = synth.uniform(102, shape_of("bkcj", ext))
    C0 = synth.uniform(103, shape_of("abij", ext))
    full = oracle.contract(spec, A, B, C0, alpha=1.5, beta=-0.5)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.integers(0, ext[ch], 50) for ch in "abij"], axis=1)
    got = oracle.contract_points(spec, A, B, pts, C0, alpha=1.5, beta=-0.5)
    assert np.array_equal(got, full[tuple(pts.T)])


def test_thread_count_does_not_change_bits():
    A = synth.uniform(111, (8, 8, 8, 8))
    B = synth.uniform(112, (8, 8, 8, 8))
    r1 = oracle.contract("abij=acik*cbkj", A, B, nthreads=1)
    r8 = oracle.contract("abij=acik*cbkj", A, B, nthreads=8)
    assert np.array_equal(r1, r8)


@pytest.mark.parametrize("spec", [
    "abij=acik*cbk",      # j only in C
    "abij=acik*cbkjj",    # repeated label within a tensor
    "abij=aik*cbkj",      # c only in B
    "abij=acik*ckj",      # b only in C
    "abij-acik*cbkj",     # no '='
    "abij=acik",          # no '*'
    "ab1j=acik*cbkj",     # bad character
])
def test_invalid_specs_are_rejected(spec):
    A = np.zeros((2, 2, 2, 2))
    B = np.zeros((2, 2, 2, 2))
    with pytest.raises(Exception):
        oracle.contract(spec, A, B)


def test_mismatched_extent_is_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.contract("ij=ik*kj", np.zeros((2, 3)), np.zeros((4, 2)))


# --------------------------------------------------------------------------
# gradient
# --------------------------------------------------------------------------

def test_gradient_specs():
    assert oracle.grad_specs("abij=acik*bkcj") == ("acik=abij*bkcj", "bkcj=acik*abij")


@pytest.mark.parametrize("spec", ["abij=acik*bkcj", "abcijk=daij*bcdk", "ajbi=kcia*cjkb", "xij=xik*xkj",
                                  "ixj=kxi*jxk"])
def test_gradient_vs_central_finite_differences(spec):
    rng = random.Random(7)
    c, a, b = oracle.split_spec(spec)
    ext = {ch: rng.randint(2, 3) for ch in set(a + b)}
    A = synth.uniform(121, shape_of(a, ext))
    B = synth.uniform(122, shape_of(b, ext))
    W = synth.uniform(123, shape_of(c, ext))
    alpha = 1.25
    loss = lambda X, Y: float(np.sum(oracle.contract(spec, X, Y, alpha=alpha) * W))
    dA, dB, _ = oracle.grad(spec, A, B, W, alpha=alpha)
    h = 1e-6
    fdA = np.zeros_like(A)
    for idx in np.ndindex(A.shape):
        Ap = A.copy(); Ap[idx] += h
        Am = A.copy(); Am[idx] -= h
        fdA[idx] = (loss(Ap, B) - loss(Am, B)) / (2 * h)
    fdB = np.zeros_like(B)
    for idx in np.ndindex(B.shape):
        Bp = B.copy(); Bp[idx] += h
        Bm = B.copy(); Bm[idx] -= h
        fdB[idx] = (loss(A, Bp) - loss(A, Bm)) / (2 * h)
    assert oracle.relerr(dA, fdA) < 1e-6
    assert oracle.relerr(dB, fdB) < 1e-6


def test_gradient_adjoint_identity():
    """<Y, contract(X, B)> == <contract_dA(Y, B), X> (dot-product test)."""
    spec = "abij=acik*bkcj"
    ext = dict(a=5, b=4, c=6, i=3, j=4, k=5)
    X = synth.uniform(131, shape_of("acik", ext))
    B = synth.uniform(132, shape_of("bkcj", ext))
    Y = synth.uniform(133, shape_of("abij", ext))
    sa, sb = oracle.grad_specs(spec)
    lhs = float(np.sum(Y * oracle.contract(spec, X, B)))
    rhs = float(np.sum(oracle.contract(sa, Y, B) * X))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    rhs2 = float(np.sum(oracle.contract(sb, X, Y) * B))
    assert abs(lhs - rhs2) <= 1e-13 * abs(lhs)


# ---- the error metric every GPU tolerance is measured with ----------------
# relerr(x, ref) = ||x - ref||_F / ||ref||_F (the normwise relative error of
# the result against the FP64 definition), with ||x - ref||_F alone when ref
# is zero.  Hand-computed values, each chosen so that one plausible slip
# changes the answer.

def test_relerr_hand_computed_pythagorean_case():
    # sqrt(3^2 + 4^2) / sqrt(0^2 + 4^2) = 5 / 4
    assert oracle.relerr([3.0, 0.0], [0.0, 4.0]) == 1.25


def test_relerr_takes_square_roots():
    # sqrt(1 + 1) / sqrt(4) = 1/sqrt(2); without the roots it would read
    # 2 / 4 = 0.5, with only the numerator's root sqrt(2) / 4
    got = oracle.relerr([1.0, 1.0], [0.0, 2.0])
    assert abs(got - 2.0 ** -0.5) < 1e-15


def test_relerr_divides_by_the_reference_norm():
    # |2 - 1| / |1| = 1, not |1 - 2| / |2| = 0.5: the denominator is ref's
    assert oracle.relerr([2.0], [1.0]) == 1.0
    assert oracle.relerr([1.0], [2.0]) == 0.5


def test_relerr_zero_reference_is_absolute():
    assert oracle.relerr([3.0, 4.0], [0.0, 0.0]) == 5.0
    assert oracle.relerr([0.0, 0.0], [0.0, 0.0]) == 0.0


def test_relerr_sums_every_element_of_a_multidimensional_array():
    # 2 x 2 arrays: one wrong element among four; norms over all of them
    x = np.array([[1.0, 2.0], [3.0, 5.0]])
    ref = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert abs(oracle.relerr(x, ref) - 1.0 / np.sqrt(30.0)) < 1e-15
    assert oracle.relerr(ref, ref) == 0.0


def test_relerr_is_scale_invariant_and_survives_large_magnitudes():
    # the squares of 1e200 overflow float64 but not the long double sums:
    # the error of a relative perturbation 1e-10 must come back as 1e-10
    ref = np.array([1e200, -1e200, 3e199])
    x = ref * (1.0 + 1e-10)
    got = oracle.relerr(x, ref)
    assert abs(got - 1e-10) < 1e-14
    assert abs(oracle.relerr(x * 1e-300, ref * 1e-300) - got) < 1e-14
