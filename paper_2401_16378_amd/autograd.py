"""Differentiable decomposition: forward and backward both run in libpauli.

For a real loss L, PyTorch hands backward grad_c = dL/dRe(c) + i dL/dIm(c)
and expects the same convention back for G.  c = 2^-N Tr(P_n G) is linear in
G (Eq. (cn_compact)), so the gradient is its adjoint applied to grad_c,
2^-N sum_n grad_c[n] P_n (every Pauli string is Hermitian); that is
pauli_decompose_backward.
"""
from __future__ import annotations

import torch


class PauliDecompose(torch.autograd.Function):
    @staticmethod
    def forward(ctx, G: torch.Tensor, algo: str = "split_bf16"):
        from . import decompose
        ctx.algo = algo
        ctx.in_dtype = G.dtype
        return decompose(G, algo=algo)

    @staticmethod
    def backward(ctx, grad_c: torch.Tensor):
        from . import decompose_backward
        g = decompose_backward(grad_c.contiguous(), algo=ctx.algo, out_dtype=ctx.in_dtype)
        return g, None


class PauliCoeffsAt(torch.autograd.Function):
    """Differentiable coefficients of a host list of Pauli strings: forward is
    pauli_coeffs_at, backward its adjoint 2^-N sum_k grad_c[k] P_{n_k}
    (pauli_coeffs_at_backward), both summed in binary64."""

    @staticmethod
    def forward(ctx, G: torch.Tensor, strings):
        from . import coeffs_at
        import numpy as np
        ctx.strings = np.asarray(strings, dtype=np.uint32).reshape(-1).copy()
        ctx.N = G.shape[-1].bit_length() - 1
        ctx.in_dtype = G.dtype
        return coeffs_at(G, ctx.strings)

    @staticmethod
    def backward(ctx, grad_c: torch.Tensor):
        from . import coeffs_at_backward
        g = coeffs_at_backward(grad_c.contiguous(), ctx.N, ctx.strings, out_dtype=ctx.in_dtype)
        return g, None
