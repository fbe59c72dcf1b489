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

from . import OversketchError, block_stride, gemm_kept, gemm_kept_prec, sketch_prepare, \
    sketch_quantize, sketch_rows, stored_count


def sketched_weight_grad(X, dY, b, N, e, seed=0, keep=None, precision="fp32", h=None,
                         sigma=None, stream=None):
    """(1/K) sum_{kept i} (S_i^T X)^T (S_i^T dY)  (d_in x d_out, float32):
    the count sketch runs over the rows (tokens) of X and dY (hashed from
    seed, or explicit tables h / sigma as in the library)."""
    import torch
    if X.dim() != 2 or dY.dim() != 2 or X.shape[0] != dY.shape[0]:
        raise OversketchError("X and dY must be 2-D with the same number of rows")
    n = X.shape[0]
    prep = sketch_prepare(n, b, N, e, seed, h=h, sigma=sigma, device=X.device, stream=stream)
    kept_keep = None if keep is None else np.asarray(keep, dtype=np.uint8)
    Xs = sketch_rows(X, b, N, e, seed=seed, keep=kept_keep, kept_only=True, h=h, sigma=sigma,
                     prep=prep, workspace=True, stream=stream)
    Ds = sketch_rows(dY, b, N, e, seed=seed, keep=kept_keep, kept_only=True, h=h, sigma=sigma,
                     prep=prep, workspace=True, stream=stream)
    nst = stored_count(N, e, kept_keep, kept_only=True)
    if precision == "fp32":
        return gemm_kept(Xs, Ds, b, stream=stream)
    QX = sketch_quantize(Xs, b, nst, precision=precision, stream=stream)
    QD = sketch_quantize(Ds, b, nst, precision=precision, stream=stream)
    return gemm_kept_prec(QX, QD, b, nst, precision=precision, stream=stream)


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
