"""Seeded synthetic inputs for the sketched product (shared by the oracle-side
tests and by the library's tests, smoke check and benchmark).

This module draws random numbers and builds input matrices of the shapes and
value distributions of the workloads; it holds none of the sketched
product's arithmetic (no hash, no sketch, no block product).

Seeding: one base seed ``s``.  Matrix entries come from NumPy's PCG64
``default_rng([s, 0])`` (A drawn first, then B); keep-masks from
``default_rng([s, 1])``.  The sketch's own random choices are not drawn here:
they are the hash key ``s`` passed to both implementations.
"""
from __future__ import annotations

import numpy as np


def data_rng(seed: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), 0])


def mask_rng(seed: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), 1])


def gaussian_pair(m: int, n: int, l: int, seed: int, dtype=np.float32):
    """A (m x n) and B (n x l) with i.i.d. N(0, 1) entries."""
    rng = data_rng(seed)
    A = rng.standard_normal((m, n), dtype=np.float32 if dtype == np.float32 else np.float64)
    B = rng.standard_normal((n, l), dtype=np.float32 if dtype == np.float32 else np.float64)
    return A.astype(dtype, copy=False), B.astype(dtype, copy=False)


def lowrank_pair(m: int, n: int, l: int, seed: int, rank: int = 64, noise: float = 0.1,
                 shared_factor: bool = True):
    """Rank-`rank` Gaussian factor products plus N(0, noise^2) noise, FP32.

    shared_factor=True:  A = U Q / sqrt(r) + noise*G_A,  B = Q^T W / sqrt(r) + noise*G_B
    (A's row space and B's column space share the factor Q, as in the paper's
    own workloads, where B = A^T or the product is a Gram matrix).
    shared_factor=False: B uses an independent factor P in place of Q^T.
    """
    rng = data_rng(seed)
    f32 = np.float32
    U = rng.standard_normal((m, rank), dtype=f32)
    Q = rng.standard_normal((rank, n), dtype=f32)
    W = rng.standard_normal((rank, l), dtype=f32)
    inv = f32(1.0 / np.sqrt(rank))
    A = U @ Q
    A *= inv
    A += f32(noise) * rng.standard_normal((m, n), dtype=f32)
    if shared_factor:
        B = Q.T @ W
    else:
        P = rng.standard_normal((n, rank), dtype=f32)
        B = P @ W
    B *= inv
    B += f32(noise) * rng.standard_normal((n, l), dtype=f32)
    return np.ascontiguousarray(A), np.ascontiguousarray(B)


def lognormal_scaled_pair(m: int, n: int, l: int, seed: int, sigma: float = 2.0):
    """A with log-normal(0, sigma) row norms, B with log-normal(0, sigma)
    column norms, directions Gaussian; FP32."""
    rng = data_rng(seed)
    f32 = np.float32
    A = rng.standard_normal((m, n), dtype=f32)
    B = rng.standard_normal((n, l), dtype=f32)
    ra = np.exp(sigma * rng.standard_normal(m)) / np.sqrt(n)
    cb = np.exp(sigma * rng.standard_normal(l)) / np.sqrt(n)
    A *= ra.astype(f32)[:, None]
    B *= cb.astype(f32)[None, :]
    return A, B


def paper_plus_matrix(m: int, n: int, dtype=np.float32):
    """A(x, y) = x + y with 1-based x in [1, m], y in [1, n] (the constant
    matrix of the paper's Lambda experiments)."""
    x = np.arange(1, m + 1, dtype=np.float64)[:, None]
    y = np.arange(1, n + 1, dtype=np.float64)[None, :]
    return (x + y).astype(dtype)


def paper_times_matrix(m: int, n: int, dtype=np.float32):
    """B(x, y) = x * y with 1-based indices (section 5.3's second factor)."""
    x = np.arange(1, m + 1, dtype=np.float64)[:, None]
    y = np.arange(1, n + 1, dtype=np.float64)[None, :]
    return (x * y).astype(dtype)


def paper_matrices_device(m: int, n: int, l: int | None = None, device="cuda"):
    """The paper's constant matrices on the device, in FP32: A(x, y) = x + y
    (m x n, exact while m + n < 2^24) and, when l is given, B(x, y) = x * y
    (n x l, each product rounded to FP32, relative error <= 2^-24), with
    1-based indices.  Also returns the index vectors (FP64, on the device)
    that define them."""
    import torch
    x = torch.arange(1, m + 1, device=device, dtype=torch.float64)
    y = torch.arange(1, n + 1, device=device, dtype=torch.float64)
    A = (x[:, None].float() + y[None, :].float())
    if l is None:
        return A, x, y
    z = torch.arange(1, l + 1, device=device, dtype=torch.float64)
    B = (y[:, None] * z[None, :]).float()
    return A, B, x, y, z


def paper_exact_products(x, y, z=None):
    """Exact FP64 products of the paper's constant matrices, from their index
    vectors (torch FP64 tensors, on any device), with the sums that the
    sketch's error formula needs.  A = x 1^T + 1 y^T (m x n), so
      - without z: B = A^T and AB = A A^T, entries n x_i x_j + (x_i + x_j) Sy
        + Syy (Sy = sum y, Syy = sum y^2);
      - with z: B = y z^T (B(k, j) = y_k z_j) and AB = (A y) z^T with
        (A y)_i = x_i Sy + Syy.
    Returns (AB, |A|_F^2, |B|_F^2, sum_k |A[:, k]|^2 |B[k, :]|^2)."""
    m, n = x.numel(), y.numel()
    Sx, Sxx = x.sum(), (x * x).sum()
    Sy, Syy = y.sum(), (y * y).sum()
    nA2 = n * Sxx + 2 * Sx * Sy + m * Syy
    colA2 = Sxx + 2 * y * Sx + m * y * y           # |A[:, k]|^2
    if z is None:
        AB = n * x[:, None] * x[None, :] + (x[:, None] + x[None, :]) * Sy + Syy
        return AB, float(nA2), float(nA2), float((colA2 * colA2).sum())
    Szz = (z * z).sum()
    Ay = x * Sy + Syy
    AB = Ay[:, None] * z[None, :]
    return AB, float(nA2), float(Syy * Szz), float((colA2 * y * y).sum() * Szz)


def random_cmask(nbI: int, nbJ: int, N: int, e: int, seed: int, drop: int | None = None):
    """Keep mask per b x b block of C, [nbI][nbJ][N+e]: every block drops
    `drop` (default e) of its N+e workers at random, independently of the
    other blocks and of the sketch (drawn from the mask stream)."""
    if drop is None:
        drop = e
    if not 0 <= drop < N + e:
        raise ValueError("must keep at least one block")
    rng = mask_rng(seed)
    cm = np.ones((nbI, nbJ, N + e), dtype=np.uint8)
    for i in range(nbI):
        for j in range(nbJ):
            if drop:
                cm[i, j, rng.choice(N + e, size=drop, replace=False)] = 0
    return cm


def random_keep(N: int, e: int, seed: int, drop: int | None = None) -> np.ndarray:
    """Keep-mask over N+e blocks with `drop` (default e) blocks dropped at
    random, independent of the sketch (drawn from the mask stream)."""
    if drop is None:
        drop = e
    if not 0 <= drop < N + e:
        raise ValueError("must keep at least one block")
    keep = np.ones(N + e, dtype=np.uint8)
    if drop:
        idx = mask_rng(seed).choice(N + e, size=drop, replace=False)
        keep[idx] = 0
    return keep


def linear_layer(tokens: int, d_in: int, d_out: int, seed: int):
    """X ~ N(0,1) (tokens x d_in), W ~ N(0, 1/d_in) (d_in x d_out), dY ~ N(0,1)."""
    rng = data_rng(seed)
    f32 = np.float32
    X = rng.standard_normal((tokens, d_in), dtype=f32)
    W = rng.standard_normal((d_in, d_out), dtype=f32) * f32(1.0 / np.sqrt(d_in))
    dY = rng.standard_normal((tokens, d_out), dtype=f32)
    return X, W, dY


def hessian_batch(count: int, seed: int, m_lo: int = 500, m_hi: int = 4000, ratio: int = 20):
    """Interior-point Hessian inputs: list of (A_k (m_k x ratio*m_k), d_k) with
    m_k uniform in [m_lo, m_hi], A_k i.i.d. N(0,1), d_k log-uniform in
    [1e-6, 1e6]."""
    rng = data_rng(seed)
    out = []
    for _ in range(count):
        mk = int(rng.integers(m_lo, m_hi + 1))
        Ak = rng.standard_normal((mk, ratio * mk), dtype=np.float32)
        dk = np.exp(rng.uniform(np.log(1e-6), np.log(1e6), size=ratio * mk)).astype(np.float32)
        out.append((Ak, dk))
    return out


def hessian_sizes(count: int, seed: int, m_lo: int = 500, m_hi: int = 4000) -> list:
    """m_k uniform in [m_lo, m_hi] for the device-generated Hessian batch
    (drawn from ``default_rng([seed, 2])``)."""
    rng = np.random.default_rng([int(seed), 2])
    return [int(v) for v in rng.integers(m_lo, m_hi + 1, size=count)]


def hessian_batch_device(count: int, seed: int, device="cuda", ratio: int = 20,
                         m_lo: int = 500, m_hi: int = 4000):
    """The interior-point Hessian batch drawn on the device (too large to
    draw on the host at full size): sizes from ``hessian_sizes``, then per
    problem A_k (m_k x ratio*m_k) i.i.d. N(0,1) and d_k log-uniform in
    [1e-6, 1e6], both from torch's device generator seeded with ``seed``.
    Returns (sizes, [A_k], [d_k])."""
    import torch
    sizes = hessian_sizes(count, seed, m_lo, m_hi)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    lo, hi = np.log(1e-6), np.log(1e6)
    As, ds = [], []
    for m in sizes:
        n = ratio * m
        As.append(torch.randn((m, n), generator=gen, device=device, dtype=torch.float32))
        u = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
        ds.append(torch.exp(lo + u * (hi - lo)).to(torch.float32))
    return sizes, As, ds
