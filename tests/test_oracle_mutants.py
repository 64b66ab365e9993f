"""Plant plausible mistakes in a copy of the oracle and check that the pins catch each.

Every mutant is a one-line edit of oracle.c (a wrong sign, a dropped term, a
wrong stride, a swapped operand, a mishandled alpha or beta, a wrong output
address).  The copy is built in a temporary folder and run in a child process
(a mutant may read out of bounds), against a battery of the independent pins:
numpy.einsum, exact integer einsum, closed forms and the DSL forms.  The real
oracle must pass the same battery.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "sign_of_product": ("s = s + prod;", "s = s - prod;"),
    "dropped_last_term": ("if (++kv[i] < tb->ext[pb->sumrow[i]]) break;",
                          "if (++kv[i] < tb->ext[pb->sumrow[i]] - (i == 0)) break;"),
    "B_uses_A_strides_for_sum": ("offB += kv[i] * tb->str[2][r];", "offB += kv[i] * tb->str[1][r];"),
    "B_uses_C_strides_for_free": ("baseB += freeval[i] * tb->str[2][r];",
                                  "baseB += freeval[i] * tb->str[0][r];"),
    "beta_value_ignored": ("double r = alpha * s;\n    if (beta != 0.0) r = r + beta * C[ac];\n    C[ac] = r;",
                           "double r = alpha * s;\n    if (beta != 0.0) r = r + C[ac];\n    C[ac] = r;"),
    "alpha_dropped": ("double r = alpha * s;\n    if (beta != 0.0) r = r + beta * C[ac];\n    C[ac] = r;",
                      "double r = s;\n    if (beta != 0.0) r = r + beta * C[ac];\n    C[ac] = r;"),
    "C_address_uses_B_strides": ("a += val[i] * pb->tb.str[0][pb->freerow[i]];",
                                 "a += val[i] * pb->tb.str[2][pb->freerow[i]];"),
    "first_term_skipped": ("double s = 0.0;\n  if (pb->nk == 0) return s;",
                           "double s = -A[baseA] * B[baseB];\n  if (pb->nk == 0) return s;"),
}

BATTERY = r'''
import ctypes, sys, random
import numpy as np
sys.path.insert(0, ROOT)
import oracle, synth
oracle._lib = oracle.bind(ctypes.CDLL(LIB))
fails = []
def check(name, ok):
    if not ok:
        fails.append(name)
def ein(spec, A, B):
    c, a, b = oracle.split_spec(spec)
    return np.einsum("%s,%s->%s" % (a, b, c), A, B)
specs = ["abij=acik*cbkj", "abij=acik*bkcj", "abcijk=daij*bcdk", "ajbi=kcia*cjkb", "ij=ik*kj", "iaj=ij*a"]
exts = [dict(a=3, b=4, c=5, d=2, i=3, j=2, k=4), dict(a=2, b=3, c=3, d=4, i=2, j=3, k=2)]
for s in specs:
    c, a, b = oracle.split_spec(s)
    for e in exts:
        A = synth.uniform(1, tuple(e[x] for x in a)); B = synth.uniform(2, tuple(e[x] for x in b))
        try:
            got = oracle.contract(s, A, B)
            check("einsum " + s, np.allclose(got, ein(s, A, B), rtol=1e-12, atol=1e-13))
            Ai = synth.integers(3, A.shape); Bi = synth.integers(4, B.shape)
            C0 = synth.integers(5, tuple(e[x] for x in c))
            got = oracle.contract(s, Ai, Bi, C0, alpha=2.0, beta=-3.0)
            ref = 2 * ein(s, Ai.astype(np.int64), Bi.astype(np.int64)) - 3 * C0.astype(np.int64)
            check("integer " + s, np.array_equal(got, ref.astype(np.float64)))
            ones = oracle.contract(s, np.ones(A.shape), np.ones(B.shape), C0, alpha=1.0, beta=1.0)
            kp = int(np.prod([e[x] for x in a if x not in c]))
            check("ones " + s, np.array_equal(ones, kp + C0))
        except Exception as ex:
            fails.append("raised %s %s" % (s, ex))
print("FAILED_PINS", len(fails))
for f in fails[:5]:
    print(f)
'''


def _run_battery(lib_path):
    code = BATTERY.replace("ROOT", repr(ROOT)).replace("LIB", repr(lib_path))
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    return p.returncode, p.stdout + p.stderr


def _build(src_text, out_dir):
    c = os.path.join(out_dir, "oracle.c")
    so = os.path.join(out_dir, "liboracle.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c99", "-shared", "-fPIC",
                    c, "-o", so], check=True)
    return so


def test_real_oracle_passes_battery(tmp_path):
    with open(SRC) as f:
        so = _build(f.read(), str(tmp_path))
    rc, out = _run_battery(so)
    assert rc == 0 and "FAILED_PINS 0" in out, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, "mutation anchor not unique/present: %s" % name
    so = _build(text.replace(old, new), str(tmp_path))
    rc, out = _run_battery(so)
    caught = rc != 0 or "FAILED_PINS 0" not in out
    assert caught, "mutant %s survived the pins:\n%s" % (name, out)
