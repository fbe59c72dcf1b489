"""Sketched linear layer: an exact forward, and a backward whose weight
gradient is OverSketch's approximate product over the token dimension.

For Y = X W (X tokens x d_in, W d_in x d_out) the weight gradient is
dW = X^T dY, a product whose inner dimension is the number of tokens.  The
backward here forms it as the sketched product of Section 4,

    dW ~= (1/K) sum_{kept i} (S_i^T X)^T (S_i^T dY),

sketching the rows (tokens) of X and of dY with the same count-sketch blocks
and multiplying the kept blocks (every step in the library's HIP kernels).
dX = dY W^T stays exact.  The sketched gradient is unbiased over the draw of
S (Lemma 2), with the second moment of Lemma 1.

Seeds: with ``seed=None`` (the default) every forward call draws a fresh
64-bit sketch key from torch's CPU generator and keeps it for its backward,
so successive training steps use independent sketches and their gradient
errors average out.  A fixed integer seed gives the same S on every call
(for tests and reproducible runs).

The exact products (forward Y and dX) are plain dense GEMMs that the layer
needs around the method, not part of it: they go to torch.matmul (the
vendor BLAS), and only the sketched product runs in this library.
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


def fresh_seed() -> int:
    """A 64-bit sketch key drawn from torch's default CPU generator (so
    torch.manual_seed makes a run reproducible)."""
    import torch
    hi = int(torch.randint(0, 2**32, (1,), dtype=torch.int64).item())
    lo = int(torch.randint(0, 2**32, (1,), dtype=torch.int64).item())
    return (hi << 32) | lo


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
                # the key this call's backward uses (drawn now when not fixed)
                key = fresh_seed() if seed is None else int(seed)
                ctx.cfg = (b, N, e, key, keep, precision, h, sigma)
                return torch.matmul(X, W)

            @staticmethod
            def backward(ctx, dY):
                X, W = ctx.saved_tensors
                b, N, e, key, keep, precision, h, sigma = ctx.cfg
                dX = None
                if ctx.needs_input_grad[0]:
                    dX = torch.matmul(dY, W.t())
                dW = None
                if ctx.needs_input_grad[1]:
                    dW = sketched_weight_grad(X, dY.contiguous(), b, N, e, seed=key, keep=keep,
                                              precision=precision, h=h, sigma=sigma).to(W.dtype)
                return dX, dW, None, None, None, None, None, None, None, None

        cls._fn = _SketchedLinear
        return cls._fn


def sketched_linear(X, W, b, N, e, seed=None, keep=None, precision="fp32", h=None, sigma=None):
    """Y = X W with the sketched weight gradient in backward.  seed=None
    draws a fresh sketch per forward call; an integer fixes it."""
    return SketchedLinearFunction.get().apply(X, W, b, N, e, seed, keep, precision, h, sigma)
