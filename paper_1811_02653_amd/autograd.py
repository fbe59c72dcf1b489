"""Sketched linear layer: an exact forward, and a backward whose weight
gradient is OverSketch's approximate product over the token dimension.

For Y = X W (X tokens x d_in, W d_in x d_out) the weight gradient is
dW = X^T dY, a product whose inner dimension is the number of tokens.  The
backward here forms it as the sketched product of Section 4,

    dW ~= (1/K) sum_{kept i} (S_i^T X)^T (S_i^T dY),

sketching the rows (tokens) of X and of dY with the same count-sketch blocks
and multiplying the kept blocks (every step in the library's HIP kernels).
dX = dY W^T stays exact.  The sketched gradient is unbiased (Lemma 2) with
the second moment of Lemma 1; a fresh seed per backward call keeps the
gradients of successive steps independent.

The exact products (forward Y and dX) are plain GEMMs and use torch.matmul.
"""
from __future__ import annotations

import numpy as np

from . import OversketchError, matmul_ex


def sketched_weight_grad(X, dY, b, N, e, seed=0, keep=None, precision="fp32", h=None,
                         sigma=None, stream=None, workspace=None):
    """(1/K) sum_{kept i} (S_i^T X)^T (S_i^T dY)  (d_in x d_out, float32):
    the count sketch runs over the rows (tokens) of X and dY (hashed from
    seed, or explicit tables h / sigma as in the library).  One library call
    (os_matmul_ex with A = X^T, read column-major, and B = dY): prepare,
    transpose-and-sketch of X and of dY (dropped blocks skipped), the block
    product in the given precision."""
    if X.dim() != 2 or dY.dim() != 2 or X.shape[0] != dY.shape[0]:
        raise OversketchError("X and dY must be 2-D with the same number of rows")
    kept_keep = None if keep is None else np.asarray(keep, dtype=np.uint8)
    return matmul_ex(X.t(), dY, b, N, e, seed=seed, keep=kept_keep, kept_only=True,
                     precision=precision, h=h, sigma=sigma, workspace=workspace, stream=stream)


class SketchedLinearFunction:
    """Factory of the torch.autograd.Function (torch is imported lazily)."""

    _fn = None

    @classmethod
    def get(cls):
        if cls._fn is not None:
            return cls._fn
        import torch

        class _SketchedLinear(torch.autograd.Function):
            @staticmethod
            def forward(ctx, X, W, b, N, e, seed, keep, precision, h, sigma):
                ctx.save_for_backward(X, W)
                ctx.cfg = (b, N, e, seed, keep, precision, h, sigma)
                return torch.matmul(X, W)

            @staticmethod
            def backward(ctx, dY):
                X, W = ctx.saved_tensors
                b, N, e, seed, keep, precision, h, sigma = ctx.cfg
                dX = None
                if ctx.needs_input_grad[0]:
                    dX = torch.matmul(dY, W.t())
                dW = None
                if ctx.needs_input_grad[1]:
                    dW = sketched_weight_grad(X, dY.contiguous(), b, N, e, seed=seed, keep=keep,
                                              precision=precision, h=h, sigma=sigma).to(W.dtype)
                return dX, dW, None, None, None, None, None, None, None, None

        cls._fn = _SketchedLinear
        return cls._fn


def sketched_linear(X, W, b, N, e, seed=0, keep=None, precision="fp32", h=None, sigma=None):
    """Y = X W with the sketched weight gradient in backward."""
    return SketchedLinearFunction.get().apply(X, W, b, N, e, seed, keep, precision, h, sigma)
