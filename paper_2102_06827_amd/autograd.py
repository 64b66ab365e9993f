"""Differentiable contraction: a hand-written backward built from the same kernels.

For C = alpha * contract(A, B) + beta * C0 and an upstream gradient dC,

    dA = alpha * contract("<A>=<C>*<B>", dC, B)
    dB = alpha * contract("<B>=<A>*<C>", A, dC)
    dC0 = beta * dC

Each gradient is itself a permuted contraction (the summation labels of one
product become free labels of the other), so it runs through the same
library call as the forward.
"""
from __future__ import annotations

import torch


def grad_specs(spec):
    s = "".join(spec.split())
    c, rhs = s.split("=")
    a, b = rhs.split("*")
    return "%s=%s*%s" % (a, c, b), "%s=%s*%s" % (b, a, c)


class ContractFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, spec, A, B, C0, alpha, beta, compute):
        from . import contract, permute
        ctx.spec, ctx.alpha, ctx.beta, ctx.compute = spec, float(alpha), float(beta), compute
        ctx.has_c0 = C0 is not None
        ctx.save_for_backward(A, B)
        C = None
        if C0 is not None and beta != 0.0:
            # a copy of C0 (the identity permutation), so the input stays untouched
            c = grad_specs(spec)[0].split("=")[1].split("*")[0]
            C = permute("%s=%s" % (c, c), C0)
        return contract(spec, A, B, C, alpha=alpha, beta=beta if C is not None else 0.0, compute=compute)

    @staticmethod
    def backward(ctx, dC):
        from . import contract, permute
        A, B = ctx.saved_tensors
        dC = dC.contiguous()
        sa, sb = grad_specs(ctx.spec)
        dA = dB = dC0 = None
        if ctx.needs_input_grad[1]:
            dA = contract(sa, dC, B, alpha=ctx.alpha, compute=ctx.compute)
        if ctx.needs_input_grad[2]:
            dB = contract(sb, A, dC, alpha=ctx.alpha, compute=ctx.compute)
        if ctx.has_c0 and ctx.needs_input_grad[3]:
            # dC0 = beta * dC through the library's permute kernel (identity
            # permutation with scale beta)
            c = sa.split("=")[1].split("*")[0]
            dC0 = permute("%s=%s" % (c, c), dC, alpha=ctx.beta)
        return None, dA, dB, dC0, None, None, None


def contract_ad(spec, A, B, C0=None, alpha=1.0, beta=0.0, compute="default"):
    """Autograd-aware contraction (gradients for A, B and C0)."""
    return ContractFn.apply(spec, A, B, C0, alpha, beta, compute)
