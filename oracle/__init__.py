"""FP64 CPU oracle for OverSketch's sketched product C ~= A S S^T B.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the library in
``paper_1811_02653_amd`` never does, and this package never imports it.

The arithmetic lives in ``oracle.c`` (plain FP64 loops, see its header for the
paper passages each function follows); this module only builds and loads it
and marshals NumPy arrays.  ``literal_*`` below are the paper's definitions
written with a dense sketch matrix (Eq. (sketch_matrix)), for tiny sizes.

Random bucket/sign choices: the paper leaves the random source open
(Algorithm "Calculating Count-sketch of a matrix A" only asks for fair signs
and uniform buckets).  Reading used here and in the library, each implemented
separately from the published definition of SplitMix64: word =
SplitMix64(seed, ctr) with ctr = (block << 40) | index, bucket =
((word >> 32) * b) >> 32, sign = -1 if word & 1 else +1.  Agreement of the
buckets with the paper's randomness is therefore "parity unpinned"; the hash
is pinned to SplitMix64's published outputs and to its distribution instead.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, u64 = ctypes.c_int64, ctypes.c_uint64
    vp = ctypes.c_void_p
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_splitmix64_nth.restype = u64
    lib.oracle_splitmix64_nth.argtypes = [u64, u64]
    lib.oracle_hash_word.restype = u64
    lib.oracle_hash_word.argtypes = [u64, u64, u64]
    lib.oracle_hash.restype = None
    lib.oracle_hash.argtypes = [u64, i64, i64, i64, vp, vp]
    lib.oracle_sketch_cols.restype = None
    lib.oracle_sketch_cols.argtypes = [vp, i64, i64, i64, vp, vp, i64, i64, vp]
    lib.oracle_sketch_rows.restype = None
    lib.oracle_sketch_rows.argtypes = [vp, i64, i64, i64, vp, vp, i64, i64, vp]
    lib.oracle_block_product.restype = i64
    lib.oracle_block_product.argtypes = [vp, vp, i64, i64, i64, i64, vp, vp]
    lib.oracle_sampled_entries.restype = i64
    lib.oracle_sampled_entries.argtypes = [vp, i64, vp, i64, i64, vp, vp, i64, i64, vp,
                                           vp, vp, i64, vp]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(x) -> np.ndarray:
    """FP64 C-contiguous copy-if-needed (FP32 -> FP64 is exact)."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().oracle_num_threads())


# ---------------------------------------------------------------------------
# Hash (reading of the random choices, see module docstring)
# ---------------------------------------------------------------------------

def splitmix64_nth(seed: int, j: int) -> int:
    """j-th output (0-based) of SplitMix64 seeded with ``seed``."""
    return int(_load().oracle_splitmix64_nth(seed & (2**64 - 1), j))


def hash_word(seed: int, blk: int, k: int) -> int:
    return int(_load().oracle_hash_word(seed & (2**64 - 1), blk, k))


def hash_tables(seed: int, nblk: int, n: int, b: int):
    """Buckets h[blk, k] in [0, b) (int32) and signs sigma[blk, k] (int8)."""
    h = np.empty((nblk, n), dtype=np.int32)
    s = np.empty((nblk, n), dtype=np.int8)
    _load().oracle_hash(seed & (2**64 - 1), nblk, n, b, _p(h), _p(s))
    return h, s


def default_keep(N: int, e: int) -> np.ndarray:
    """Mask used when none is given: blocks [0, N) kept, the e extra dropped."""
    keep = np.zeros(N + e, dtype=np.uint8)
    keep[:N] = 1
    return keep


# ---------------------------------------------------------------------------
# Sketch and product (oracle.c)
# ---------------------------------------------------------------------------

def _check_tables(h, s, n, b):
    h = np.ascontiguousarray(h, dtype=np.int32)
    s = np.ascontiguousarray(s, dtype=np.int8)
    if h.ndim != 2 or h.shape != s.shape or h.shape[1] != n:
        raise ValueError("hash tables must be [nblk, n] with n = %d" % n)
    if h.size and (h.min() < 0 or h.max() >= b):
        raise ValueError("bucket outside [0, b)")
    if s.size and not np.all(np.abs(s.astype(np.int32)) == 1):
        raise ValueError("signs must be +-1")
    return h, s


def sketch_cols(A, h, sigma, b: int) -> np.ndarray:
    """A_tilde = [A S_0, ..., A S_{nblk-1}] (m x nblk*b, FP64, unscaled)."""
    A = _f64(A)
    m, n = A.shape
    h, s = _check_tables(h, sigma, n, b)
    nblk = h.shape[0]
    out = np.empty((m, nblk * b), dtype=np.float64)
    _load().oracle_sketch_cols(_p(A), m, n, n, _p(h), _p(s), nblk, b, _p(out))
    return out


def sketch_rows(B, h, sigma, b: int) -> np.ndarray:
    """B_tilde = [S_0^T B; ...; S_{nblk-1}^T B] (nblk*b x l, FP64, unscaled)."""
    B = _f64(B)
    n, l = B.shape
    h, s = _check_tables(h, sigma, n, b)
    nblk = h.shape[0]
    out = np.empty((nblk * b, l), dtype=np.float64)
    _load().oracle_sketch_rows(_p(B), n, l, l, _p(h), _p(s), nblk, b, _p(out))
    return out


def block_product(At, Bt, b: int, keep) -> np.ndarray:
    """C = (1/K) sum_{kept i} At_i Bt_i (FP64)."""
    At, Bt = _f64(At), _f64(Bt)
    m, z = At.shape
    z2, l = Bt.shape
    if z != z2 or z % b:
        raise ValueError("sketch widths disagree")
    nblk = z // b
    keep = np.ascontiguousarray(keep, dtype=np.uint8)
    if keep.shape != (nblk,):
        raise ValueError("keep mask must have one entry per block")
    C = np.empty((m, l), dtype=np.float64)
    K = _load().oracle_block_product(_p(At), _p(Bt), m, l, b, nblk, _p(keep), _p(C))
    if K == 0:
        raise ValueError("keep mask keeps no block")
    return C


def sketched_matmul(A, B, b: int, N: int, e: int, seed: int = 0, keep=None,
                    h=None, sigma=None) -> np.ndarray:
    """OverSketch product (Algorithm "OverSketch"): sketch A's columns and B's
    rows with all N+e blocks, then combine the kept blocks with weight 1/K."""
    A, B = _f64(A), _f64(B)
    n = A.shape[1]
    if B.shape[0] != n:
        raise ValueError("inner dimensions differ")
    if h is None:
        h, sigma = hash_tables(seed, N + e, n, b)
    if keep is None:
        keep = default_keep(N, e)
    At = sketch_cols(A, h, sigma, b)
    Bt = sketch_rows(B, h, sigma, b)
    return block_product(At, Bt, b, keep)


def sampled_entries(A, B, rows, cols, b: int, N: int, e: int, seed: int = 0,
                    keep=None, h=None, sigma=None) -> np.ndarray:
    """C[rows[t], cols[t]] by the same definition, one entry at a time."""
    A = np.asarray(A)
    B = np.asarray(B)
    m, n = A.shape
    n2, l = B.shape
    if n2 != n:
        raise ValueError("inner dimensions differ")
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape or rows.ndim != 1:
        raise ValueError("rows and cols must be 1-D of equal length")
    if rows.size and (rows.min() < 0 or rows.max() >= m or cols.min() < 0 or cols.max() >= l):
        raise ValueError("sample index out of range")
    if h is None:
        h, sigma = hash_tables(seed, N + e, n, b)
    h, s = _check_tables(h, sigma, n, b)
    nblk = h.shape[0]
    if keep is None:
        keep = default_keep(N, e)
    keep = np.ascontiguousarray(keep, dtype=np.uint8)
    # Only the sampled rows of A and columns of B are needed; convert those.
    ur, inv_r = np.unique(rows, return_inverse=True)
    uc, inv_c = np.unique(cols, return_inverse=True)
    Asub = _f64(A[ur, :])
    Bsub = _f64(B[:, uc])
    out = np.empty(rows.size, dtype=np.float64)
    K = _load().oracle_sampled_entries(_p(Asub), n, _p(Bsub), uc.size, n, _p(h), _p(s),
                                       nblk, b, _p(keep), _p(np.ascontiguousarray(inv_r, np.int64)),
                                       _p(np.ascontiguousarray(inv_c, np.int64)), rows.size, _p(out))
    if K == 0:
        raise ValueError("keep mask keeps no block")
    return out


def sketched_matmul_cmask(A, B, b: int, N: int, e: int, cmask, seed: int = 0,
                          h=None, sigma=None) -> np.ndarray:
    """OverSketch product with a keep mask per b x b block of C (Algorithm
    "OverSketch": each block of C is assembled from the workers that
    returned for it).  cmask[I, J, i] != 0 keeps sketch block i for C block
    (I, J) (rows I*b.., columns J*b.., the last ones partial):
        C_IJ = (1/K_IJ) sum_{kept i} (A_I S_i)(S_i^T B_J),
    K_IJ its kept count; a block that keeps none is zero."""
    A, B = _f64(A), _f64(B)
    m, n = A.shape
    l = B.shape[1]
    if B.shape[0] != n:
        raise ValueError("inner dimensions differ")
    cmask = np.asarray(cmask, dtype=np.uint8)
    nbI, nbJ = -(-m // b), -(-l // b)
    if cmask.shape != (nbI, nbJ, N + e):
        raise ValueError("cmask must be [ceil(m/b)][ceil(l/b)][N+e]")
    if h is None:
        h, sigma = hash_tables(seed, N + e, n, b)
    At = sketch_cols(A, h, sigma, b)
    Bt = sketch_rows(B, h, sigma, b)
    C = np.zeros((m, l))
    for I in range(nbI):
        for J in range(nbJ):
            if cmask[I, J].any():
                r = slice(I * b, min(m, (I + 1) * b))
                c = slice(J * b, min(l, (J + 1) * b))
                C[r, c] = block_product(At[r], Bt[:, c], b, cmask[I, J])
    return C


def sketched_gram(A, d, b: int, N: int, e: int, seed: int = 0, keep=None,
                  h=None, sigma=None) -> np.ndarray:
    """Sketched Hessian of the log-barrier interior-point method (Section 5.2,
    Eq. (int_point) and the Hessian after it): the Hessian's square root is
    the constraint matrix with row i scaled by 1/|b_i - a_i x|, and the
    Hessian is approximated by the Gram matrix of its sketch.  Here A (m x n)
    is the constraint matrix transposed and d (n, >= 0) the squared scales
    1/(b_i - a_i x)^2 (None = ones), so the result is the OverSketch product
    of W = A diag(sqrt(d)) with W^T:
        H = (1/K) sum_{kept i} (W S_i)(S_i^T W^T)."""
    A = _f64(A)
    if d is not None:
        d = np.asarray(d, dtype=np.float64).reshape(-1)
        if d.shape[0] != A.shape[1] or np.any(d < 0):
            raise ValueError("d must hold n nonnegative weights")
        A = A * np.sqrt(d)[None, :]
    return sketched_matmul(A, np.ascontiguousarray(A.T), b, N, e, seed=seed, keep=keep,
                           h=h, sigma=sigma)


# ---------------------------------------------------------------------------
# Literal definitions with a dense sketch matrix (tiny sizes only)
# ---------------------------------------------------------------------------

def literal_blocks(h, sigma, b: int) -> np.ndarray:
    """Dense [S_0, ..., S_{nblk-1}] (n x nblk*b): S_i[k, h_i(k)] = sigma_i(k),
    every other entry zero (a count-sketch matrix, Eq. (count_sketch_example))."""
    h = np.asarray(h)
    sigma = np.asarray(sigma)
    nblk, n = h.shape
    S = np.zeros((n, nblk * b), dtype=np.float64)
    for i in range(nblk):
        for k in range(n):
            S[k, i * b + int(h[i, k])] = float(sigma[i, k])
    return S


def literal_product(A, B, h, sigma, b: int, N: int, keep) -> np.ndarray:
    """A S_K S_K^T B with S = N^{-1/2} (S_1, ..., S_{N+e}) (Eq. (sketch_matrix))
    restricted to the kept blocks, evaluated with dense matrices."""
    S = literal_blocks(h, sigma, b) / np.sqrt(N)
    cols = np.concatenate([np.arange(i * b, (i + 1) * b) for i in np.flatnonzero(keep)])
    SK = S[:, cols]
    return (_f64(A) @ SK) @ (SK.T @ _f64(B))


# ---------------------------------------------------------------------------
# Reduced-precision operands (the precision direction of the block product;
# not in the paper, whose products are FP64)
# ---------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """FP32 -> BF16 with round-to-nearest-even, returned as FP32 values.

    BF16 is the upper 16 bits of an FP32 word (1 sign, 8 exponent, 7
    fraction bits).  Round to nearest even on the dropped 16 bits: add
    0x7FFF plus the lowest kept bit, then clear the dropped bits.  Overflow
    carries into the exponent (to infinity above the largest BF16), as the
    rounding rule requires.  NaNs stay NaN (made quiet)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + keep_lsb) >> np.uint64(16)) << np.uint64(16)
    r = r.astype(np.uint32)
    nan = np.isnan(x)
    if nan.any():
        r[nan] = (x.view(np.uint32)[nan] & np.uint32(0xFFFF0000)) | np.uint32(0x00400000)
    return r.view(np.float32).reshape(x.shape)


def bf16_split(x):
    """(hi, lo) with hi = bf16(x) and lo = bf16(x - hi), FP32 values; x - hi is
    exact in FP32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi, lo


# FP8 E4M3 (OCP): 1 sign, 4 exponent bits (bias 7), 3 fraction bits; no
# infinities; the all-ones exponent with fraction 111 is NaN, so the largest
# finite magnitude is 1.75 * 2^8 = 448; subnormals are m * 2^-9, m = 1..7.
E4M3_MAX = 448.0


def e4m3_values() -> np.ndarray:
    """The 127 non-negative finite E4M3 magnitudes, indexed by their 7-bit
    code (exponent << 3 | fraction)."""
    v = np.empty(127)
    for code in range(127):
        e, m = code >> 3, code & 7
        v[code] = m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
    return v


def e4m3_round(y) -> np.ndarray:
    """Nearest E4M3 value to each y (|y| <= 448), ties to the even code."""
    y = np.asarray(y, dtype=np.float64)
    vals = e4m3_values()
    a = np.abs(y)
    hi = np.clip(np.searchsorted(vals, a), 1, 126)
    lo = hi - 1
    dlo, dhi = a - vals[lo], vals[hi] - a
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo % 2 == 0, lo, hi)))
    return np.sign(y) * vals[pick]


def e8m0_scale_exponent(amax: float) -> int:
    """The smallest integer s with amax <= 448 * 2^s, clamped to [-127, 127]
    (the power-of-two scale of a block; E8M0 stores s + 127)."""
    if not amax > 0:
        return -127
    s = int(np.floor(np.log2(amax / E4M3_MAX)))
    while amax > E4M3_MAX * 2.0 ** s:
        s += 1
    while amax <= E4M3_MAX * 2.0 ** (s - 1):
        s -= 1
    return max(-127, min(127, s))


def fp8_block_quantize(x, block: int = 32):
    """Per row, per `block` consecutive values: the scale exponent s of the
    block and the dequantized values e4m3_round(x * 2^-s) * 2^s.  Returns
    (values (FP64, same shape as x), exponents (rows x cols/block))."""
    x = np.asarray(x, dtype=np.float64)
    rows, cols = x.shape
    if cols % block:
        raise ValueError("columns must be a multiple of the block")
    xb = x.reshape(rows, cols // block, block)
    amax = np.abs(xb).max(axis=2)
    s = np.vectorize(e8m0_scale_exponent, otypes=[np.int64])(amax)
    sc = np.ldexp(1.0, s)[:, :, None]
    q = e4m3_round(xb / sc) * sc
    return q.reshape(rows, cols), s


def fp8_split(x, block: int = 32):
    """(hi, lo): hi the block-quantized x, lo the block-quantized residual
    x - hi (each with its own scales), FP64 values."""
    hi, _ = fp8_block_quantize(x, block)
    lo, _ = fp8_block_quantize(np.asarray(x, np.float64) - hi, block)
    return hi, lo


# ---------------------------------------------------------------------------
# Error measures (Definition of (eps, theta)-accuracy; Fig. 5b's metric)
# ---------------------------------------------------------------------------

def frob2(X) -> float:
    X = np.asarray(X, dtype=np.float64)
    return float(np.sum(X * X))


def rel_frob(X, Y) -> float:
    """||X - Y||_F / ||Y||_F in FP64."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    den = np.sqrt(frob2(Y))
    return float(np.sqrt(frob2(X - Y)) / den) if den > 0 else float(np.sqrt(frob2(X)))


def normalised_err2(C, A, B, AB=None) -> float:
    """||C - AB||_F^2 / (||A||_F^2 ||B||_F^2)."""
    A = _f64(A)
    B = _f64(B)
    if AB is None:
        AB = A @ B
    return frob2(np.asarray(C, np.float64) - AB) / (frob2(A) * frob2(B))
