"""Helpers shared by the GPU parity tests: seeded inputs and oracle comparison."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5, "split_bf16": 1e-9, "split_bf16x3": 1e-5, "split_fp16x2": 1e-5}


def torch_dev(x, dtype):
    import torch
    x = np.asarray(x)
    return torch.from_numpy(np.ascontiguousarray(x).reshape(x.shape)).to(dtype=dtype, device="cuda")


def to_np(t):
    return t.detach().double().cpu().numpy()


def shape_of(labels, ext):
    return tuple(ext[ch] for ch in labels)


def inputs(spec, ext, seed, kind="uniform", beta=False):
    c, a, b = oracle.split_spec(spec)
    if kind == "integer":
        gen = synth.integers
    elif kind == "normal":
        gen = synth.normal
    else:
        gen = synth.uniform
    A = gen(seed + 1, shape_of(a, ext))
    B = gen(seed + 2, shape_of(b, ext))
    C0 = gen(seed + 3, shape_of(c, ext)) if beta else None
    return A, B, C0


def print_case(*parts):
    """Name the case on stdout before a GPU step (flushed, so a fault still shows it)."""
    print("[case]", *parts, flush=True)
