"""Host sanitizer runs (no GPU): the planner (plan.cpp, chain.cpp) and the
oracle (oracle.c) built with -fsanitize=address,undefined by the host
compilers (g++ / gcc; no device code is involved) and driven over random
and edge-case contractions.  Any sanitizer report fails the test."""
import os
import random
import shutil
import subprocess

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_06827_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="host compilers not found")


def _build(tmp_path, name, cmd):
    exe = str(tmp_path / name)
    p = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
    return exe


def _run(exe, text):
    p = subprocess.run([exe], input=text, capture_output=True, text=True, env=ENV, timeout=300)
    bad = ("runtime error", "AddressSanitizer", "LeakSanitizer")
    assert p.returncode == 0 and not any(b in p.stderr for b in bad), p.stderr[-4000:]
    return p.stdout


def _random_spec(rng, max_per_class=3, batch=False):
    letters = list("abcdefghijklmnopqrstuvwxyzABCDEFGHIJ")
    rng.shuffle(letters)
    nm, nn, nk = rng.randint(0, max_per_class), rng.randint(0, max_per_class), rng.randint(0, max_per_class)
    nx = rng.randint(0, 2) if batch else 0
    m = letters[:nm]
    n = letters[nm:nm + nn]
    k = letters[nm + nn:nm + nn + nk]
    x = letters[nm + nn + nk:nm + nn + nk + nx]
    a, b, c = m + k + x, k + n + x, m + n + x
    for t in (a, b, c):
        rng.shuffle(t)
    return "%s=%s*%s" % ("".join(c), "".join(a), "".join(b))


def _labels(spec):
    seen = []
    for ch in spec.replace("=", "").replace("*", ""):
        if ch not in seen:
            seen.append(ch)
    return seen


def test_planner_under_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "planner", ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                       os.path.join(HERE, "planner_driver.cpp"), os.path.join(CSRC, "plan.cpp"),
                                       os.path.join(CSRC, "permute_shape.cpp"), os.path.join(CSRC, "chain.cpp")])
    rng = random.Random(2024)
    lines = []
    fixed = ["abij=acik*cbkj", "abij=acik*bkcj", "abcijk=daij*bcdk", "abij=abcd*cdij", "abij=ijcd*cdab",
             "abij=ciak*bkjc", "ajbi=kcia*cjkb", "ij=ik*kj", "=ab*ab", "iaj=ij*a", "bij=bik*bkj", "ijk=ijk*ijk"]
    for spec in fixed:
        for e in (1, 2, 3, 16):
            lines.append("p %s %s" % (spec, " ".join([str(e)] * len(_labels(spec)))))
    for _ in range(400):
        spec = _random_spec(rng, batch=rng.random() < 0.3)
        ext = [rng.choice([0, 1, 2, 3, 5, 8, 17]) for _ in _labels(spec)]
        lines.append("p %s %s" % (spec, " ".join(map(str, ext))))
    # explicit strides: every tensor a strided view (stride x2 on its last label)
    for _ in range(100):
        spec = _random_spec(rng)
        labs = _labels(spec)
        ext = {ch: rng.randint(1, 5) for ch in labs}
        c, ab = spec.split("=")
        a, b = ab.split("*")

        def strides(t):
            s, x = [], 2
            for ch in reversed(t):
                s.append(x)
                x *= ext[ch] + 1
            return list(reversed(s))
        lines.append("s %s %s | %s | %s | %s" % (spec, " ".join(str(ext[ch]) for ch in labs),
                                                 " ".join(map(str, strides(a))), " ".join(map(str, strides(b))),
                                                 " ".join(map(str, strides(c)))))
    # malformed and out-of-range input
    for bad in ("abij=acik*cbk 2 2 2 2 2 2", "abij=acik*cbkjj 2 2 2 2 2 2", "ab1j=acik*cbkj 2 2 2 2 2 2",
                "abij=acik 2 2 2 2", "abij=acik*cbkj 2 2 -1 2 2 2", "abcdefghijklm=abcdefghijklmz*z " + "1 " * 14,
                "ab=ak*kb 4611686018427387904 4 4"):
        lines.append("p " + bad)
    # chains: the shapes of Table 1 and random ones
    for spec, ext in (("ia=cdmn*inad*mc", [32, 96, 96, 96, 32, 32]), ("ia=cdmn*id*na*mc", [32, 96, 96, 96, 32, 32]),
                      ("abij=mnef*am*fn*ebij", [96, 96, 32, 32, 32, 32, 96, 96])):
        lines.append("c %s %s" % (spec, " ".join(map(str, ext))))
    for bad in ("abc=ab", "a=ab*bc*cd*de*ef*fg*gh*hi*ij", "ab=a*b"):
        lines.append("c %s %s" % (bad, " ".join(["3"] * len(_labels(bad)))))
    out = _run(exe, "\n".join(lines) + "\n")
    assert out.count("\n") >= len(lines)


def test_oracle_under_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "oracle", ["gcc", "-std=c99", "-ffp-contract=off", *SAN, os.path.join(HERE, "oracle_driver.c"),
                                      os.path.join(os.path.dirname(oracle.__file__), "oracle.c"), "-lm"])
    rng = random.Random(7)
    lines = []
    for i in range(300):
        spec = _random_spec(rng, batch=rng.random() < 0.3)
        ext = {ch: rng.randint(0 if i % 10 == 0 else 1, 4) for ch in _labels(spec)}
        c, ab = spec.split("=")
        a, b = ab.split("*")
        alpha, beta = rng.choice([(1.0, 0.0), (0.0, 2.0), (-1.5, 0.5)])

        def dims(t):
            return "%d %s" % (len(t), " ".join(str(ext[ch]) for ch in t))
        lines.append("%s %r %r %s %s %s" % (spec, alpha, beta, dims(a), dims(b), dims(c)))
    out = _run(exe, "\n".join(lines) + "\n")
    last = out.strip().splitlines()[-1].split()
    assert last[0] == "cases" and int(last[1]) == 300
    assert float(last[3]) == 0.0   # integer inputs: contraction == brute force == points, exactly
