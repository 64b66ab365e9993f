"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds random-number generation and value layouts only -- none of
the contraction's arithmetic -- so that the oracle and the GPU path can be fed
identical inputs without sharing code.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  Draw i (0-based) of a stream with seed s is
mix(s + (i + 1) * 0x9E3779B97F4A7C15 mod 2**64), where mix is the published
finaliser (xor-shift 30, multiply 0xBF58476D1CE4E5B9, xor-shift 27, multiply
0x94D049BB133111EB, xor-shift 31).

Values are produced in row-major order of the tensor's label string, in FP64;
FP32 storage rounds them to nearest-even afterwards.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """n consecutive SplitMix64 outputs (uint64) of the stream `seed`, from draw `start`."""
    i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def unit(seed: int, n: int) -> np.ndarray:
    """Uniform [0, 1) doubles: (z >> 11) * 2**-53."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    n = int(np.prod(shape, dtype=np.int64))
    u = unit(seed, n)
    return (lo + (hi - lo) * u).reshape(shape)


def normal(seed: int, shape) -> np.ndarray:
    """Standard normal by Box-Muller (cosine branch), two draws per value.

    u1 = ((z >> 11) + 1) * 2**-53 lies in (0, 1], so log(u1) is finite.
    """
    n = int(np.prod(shape, dtype=np.int64))
    z = splitmix64(seed, 2 * n) >> np.uint64(11)
    u1 = (z[0::2].astype(np.float64) + 1.0) * (2.0 ** -53)
    u2 = z[1::2].astype(np.float64) * (2.0 ** -53)
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).reshape(shape)


def integers(seed: int, shape, lo: int = -3, hi: int = 3) -> np.ndarray:
    """Uniform integers in [lo, hi] stored as doubles: (z >> 32) mod (hi-lo+1) + lo."""
    n = int(np.prod(shape, dtype=np.int64))
    z = splitmix64(seed, n) >> np.uint64(32)
    span = np.uint64(hi - lo + 1)
    return ((z % span).astype(np.int64) + lo).astype(np.float64).reshape(shape)


def decay_envelope(labels: str, shape, virtual: str, occupied: str, scale: float = 8.0) -> np.ndarray:
    """exp(-gap/scale) with gap = |v1 - v2| + |o1 - o2| over the tensor's labels.

    v1, v2 are the values of the tensor's two virtual labels (first two of
    `virtual` present in `labels`, in the tensor's order) and o1, o2 likewise
    for occupied labels; a missing pair contributes 0.  This is the
    index-gap decay of coupled-cluster amplitudes used by the CCSD-like
    workload.
    """
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    gap = np.zeros(shape, dtype=np.float64)
    for group in (virtual, occupied):
        pos = [p for p, ch in enumerate(labels) if ch in group]
        if len(pos) >= 2:
            gap = gap + np.abs(grids[pos[0]] - grids[pos[1]])
    return np.exp(-gap / scale)


def decayed_normal(seed: int, labels: str, shape, virtual: str, occupied: str) -> np.ndarray:
    return normal(seed, shape) * decay_envelope(labels, shape, virtual, occupied)


def config_seed(config: int, role: str) -> int:
    """Stream seed: 1000 * config + {A: 1, B: 2, C0: 3, W: 4}."""
    return 1000 * int(config) + {"A": 1, "B": 2, "C0": 3, "W": 4}[role]


def to_dtype(x: np.ndarray, dtype) -> np.ndarray:
    """Round FP64 values to the storage dtype (numpy casts round to nearest-even)."""
    return np.ascontiguousarray(x.astype(dtype))


# --------------------------------------------------------------------------
# the same streams generated with torch (any device), for inputs too large to
# draw on the host; bit-identical to the numpy functions above
# --------------------------------------------------------------------------

def _u64_const(x):
    """A uint64 constant as the int64 with the same bits."""
    return x - (1 << 64) if x >= (1 << 63) else x


def splitmix64_torch(seed: int, n: int, device="cpu", start: int = 0):
    import torch
    i = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    z = (i * _u64_const(0x9E3779B97F4A7C15)) + _u64_const(seed & ((1 << 64) - 1))
    # logical right shifts of int64 bit patterns: arithmetic shift, then mask
    z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * _u64_const(0xBF58476D1CE4E5B9)
    z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * _u64_const(0x94D049BB133111EB)
    z = z ^ ((z >> 31) & ((1 << 33) - 1))
    return z


def uniform_torch(seed: int, shape, dtype=None, device="cpu", lo: float = -1.0, hi: float = 1.0):
    import torch
    n = 1
    for s in shape:
        n *= int(s)
    z = splitmix64_torch(seed, n, device)
    u = ((z >> 11) & ((1 << 53) - 1)).to(torch.float64) * (2.0 ** -53)
    x = (lo + (hi - lo) * u).reshape(tuple(shape))
    return x if dtype is None else x.to(dtype)


def integers_torch(seed: int, shape, dtype=None, device="cpu", lo: int = -3, hi: int = 3):
    """The values of integers() drawn with torch on any device."""
    import torch
    n = 1
    for s in shape:
        n *= int(s)
    z = (splitmix64_torch(seed, n, device) >> 32) & ((1 << 32) - 1)
    x = (z % (hi - lo + 1) + lo).to(torch.float64).reshape(tuple(shape))
    return x if dtype is None else x.to(dtype)


# the six contraction patterns of the batched workload: 4D = 4D x 4D, output
# labels a, b, i, j split two and two between A and B, two summation labels
BATCH_PATTERNS = [
    "abij=acik*cbkj",   # block-interleaved
    "abij=acik*bkcj",   # the CCSD-like pattern
    "abij=abcd*cdij",   # a plain matrix product
    "abij=ijcd*cdab",   # transposed-output product
    "abij=ciak*bkjc",   # summation labels at both ends of A
    "ajbi=kcia*cjkb",   # A's unit label is free; C's unit label comes from A
]


def batch_problems(n: int, seed: int, extents=(8, 16, 24, 32, 40, 48, 56, 64)):
    """n problems: pattern drawn uniformly from BATCH_PATTERNS, every label's
    extent drawn independently from `extents` (SplitMix64 stream `seed`)."""
    z = splitmix64(seed, 8 * n)
    out = []
    for i in range(n):
        w = z[8 * i: 8 * i + 8]
        spec = BATCH_PATTERNS[int(w[0] % np.uint64(len(BATCH_PATTERNS)))]
        labels = sorted(set(spec) - {"=", "*"})
        ext = {ch: int(extents[int(w[1 + q] % np.uint64(len(extents)))]) for q, ch in enumerate(labels)}
        out.append((spec, ext))
    return out


def batch_check_sample(problems, n_sample: int = 128, seed: int = 5005, heaviest: int = 20,
                       small_flops: float = 2.0 ** 24):
    """Indices of the batched problems checked in full against the oracle: a
    seeded sample of n_sample problems, every problem of at most small_flops
    forward FLOPs (2 x the product of its extents) and the `heaviest` largest
    ones, sorted."""
    flops = []
    for _, ext in problems:
        p = 1
        for v in ext.values():
            p *= int(v)
        flops.append(2.0 * p)
    n = len(problems)
    chosen = [int(i) for i in np.argsort(splitmix64(seed, n), kind="stable")[:n_sample]]   # seeded permutation
    out = set(chosen)
    out |= {i for i in range(n) if flops[i] <= small_flops}
    out |= set(int(i) for i in np.argsort(np.array(flops), kind="stable")[::-1][:heaviest])
    return sorted(out)
