"""MI355X (gfx950) OverSketch: the sketched matrix product C ~= A S S^T B.

Python binding of ``liboversketch.so`` (see ``include/oversketch.h``).  This
module only marshals arguments: torch tensors supply device pointers and the
current HIP stream, NumPy arrays supply host keep-masks, and every step of the
computation runs in the library's HIP kernels.  If the library is not built,
every call raises ``OversketchError``; there is no fallback path.

Build with ``python -m paper_1811_02653_amd.build``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "OversketchError", "lib", "block_stride", "hash_fill", "sketch_prepare", "bucket_order",
    "list_entries",
    "sketch_cols",
    "sketch_rows", "sketch_rows_workspace_bytes", "gemm_kept", "matmul", "workspace_bytes",
    "stored_count", "PRECISIONS", "block_stride_prec", "quantized_row", "sketch_quantize",
    "gemm_kept_prec", "gemm_kept_cmask", "matmul_cmask", "matmul_ex", "GramBatch",
    "matmul_noalloc", "noalloc_scratch_bytes",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboversketch.so")

OS_OK = 0
OS_MAX_BLOCKS = 256
OS_MAX_B = 8192

# operand precisions of the block product (OS_PREC_* in oversketch.h)
PRECISIONS = {"fp32": 0, "bf16": 1, "bf16x3": 2, "fp8": 3, "fp8x3": 4}


class OversketchError(RuntimeError):
    """Raised for a non-OS_OK status or when the HIP library is missing."""

    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


class _Sketch(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("b", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("e", ctypes.c_int32),
        ("h", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p),
    ]


class _GramProblem(ctypes.Structure):
    _fields_ = [
        ("sk", _Sketch),
        ("A", ctypes.c_void_p),
        ("lda", ctypes.c_int64),
        ("d", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("keep", ctypes.c_void_p),
        ("H", ctypes.c_void_p),
        ("ldh", ctypes.c_int64),
    ]


class _GramCandidate(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("grid", ctypes.c_int32), ("ms", ctypes.c_float)]


_lib = None


def lib():
    """The loaded liboversketch.so (raises OversketchError if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OversketchError("liboversketch.so is not built (python -m paper_1811_02653_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, vp, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
    sk = ctypes.POINTER(_Sketch)
    L.os_status_string.restype = ctypes.c_char_p
    L.os_status_string.argtypes = [ctypes.c_int]
    L.os_last_hip_error.restype = ctypes.c_int
    L.os_last_hip_error.argtypes = []
    L.os_block_stride.restype = i32
    L.os_block_stride.argtypes = [i32]
    L.os_hash_fill.restype = ctypes.c_int
    L.os_hash_fill.argtypes = [sk, i64, vp, vp, vp]
    L.os_sketch_prepare_bytes.restype = sz
    L.os_sketch_prepare_bytes.argtypes = [sk, i64]
    L.os_sketch_prepare.restype = ctypes.c_int
    L.os_sketch_prepare.argtypes = [sk, i64, vp, sz, vp]
    L.os_sketch_prepare_ex.restype = ctypes.c_int
    L.os_sketch_prepare_ex.argtypes = [sk, i64, ctypes.c_int, vp, sz, vp]
    L.os_sketch_list_entries.restype = ctypes.c_int
    L.os_sketch_list_entries.argtypes = [sk, i64, vp, sz, vp, vp, vp]
    L.os_sketch_bucket_order.restype = ctypes.c_int
    L.os_sketch_bucket_order.argtypes = [sk, i64, vp, sz, vp, vp]
    L.os_sketch_cols.restype = ctypes.c_int
    L.os_sketch_cols.argtypes = [sk, vp, sz, vp, i64, i64, i64, vp, ctypes.c_int, vp, i64, vp]
    L.os_sketch_rows.restype = ctypes.c_int
    L.os_sketch_rows.argtypes = [sk, vp, sz, vp, i64, i64, i64, vp, ctypes.c_int, vp, i64, vp, sz,
                                 vp]
    L.os_sketch_rows_workspace_bytes.restype = sz
    L.os_sketch_rows_workspace_bytes.argtypes = [i64, i64]
    L.os_sketch_rows_ex.restype = ctypes.c_int
    L.os_sketch_rows_ex.argtypes = [sk, vp, sz, vp, ctypes.c_int, i64, i64, i64, vp, ctypes.c_int,
                                    vp, i64, vp, sz, vp]
    L.os_gemm_kept.restype = ctypes.c_int
    L.os_gemm_kept.argtypes = [vp, i64, vp, i64, i64, i64, i32, i32, vp, vp, i64, vp]
    L.os_matmul_workspace_bytes.restype = sz
    L.os_matmul_workspace_bytes.argtypes = [sk, i64, i64, i64, ctypes.c_int]
    L.os_matmul.restype = ctypes.c_int
    L.os_matmul.argtypes = [sk, vp, i64, vp, i64, ctypes.c_int, i64, i64, i64, vp, ctypes.c_int,
                            vp, i64, vp, sz, vp]
    L.os_block_stride_prec.restype = i32
    L.os_block_stride_prec.argtypes = [i32, ctypes.c_int]
    L.os_quantized_row.restype = i64
    L.os_quantized_row.argtypes = [i32, i32, ctypes.c_int]
    L.os_sketch_quantize.restype = ctypes.c_int
    L.os_sketch_quantize.argtypes = [vp, i64, i64, i32, i32, ctypes.c_int, vp, i64, vp]
    L.os_gemm_kept_prec.restype = ctypes.c_int
    L.os_gemm_kept_prec.argtypes = [vp, i64, vp, i64, i64, i64, i32, i32, vp, ctypes.c_int, vp,
                                    i64, vp]
    L.os_gemm_kept_cmask.restype = ctypes.c_int
    L.os_gemm_kept_cmask.argtypes = [vp, i64, vp, i64, i64, i64, i32, i32, vp, vp, i64, vp]
    L.os_matmul_cmask.restype = ctypes.c_int
    L.os_matmul_cmask.argtypes = [sk, vp, i64, vp, i64, ctypes.c_int, i64, i64, i64, vp, vp, i64,
                                  vp, sz, vp]
    L.os_matmul_prec_workspace_bytes.restype = sz
    L.os_matmul_prec_workspace_bytes.argtypes = [sk, i64, i64, i64, ctypes.c_int, ctypes.c_int]
    L.os_matmul_prec.restype = ctypes.c_int
    L.os_matmul_prec.argtypes = [sk, vp, i64, vp, i64, ctypes.c_int, i64, i64, i64, vp,
                                 ctypes.c_int, ctypes.c_int, vp, i64, vp, sz, vp]
    L.os_noalloc_scratch_bytes.restype = sz
    L.os_noalloc_scratch_bytes.argtypes = []
    L.os_matmul_noalloc.restype = ctypes.c_int
    L.os_matmul_noalloc.argtypes = [sk, vp, i64, vp, i64, ctypes.c_int, i64, i64, i64, vp,
                                    ctypes.c_int, ctypes.c_int, vp, i64, vp]
    L.os_matmul_ex_workspace_bytes.restype = sz
    L.os_matmul_ex_workspace_bytes.argtypes = [sk, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int]
    L.os_matmul_ex.restype = ctypes.c_int
    L.os_matmul_ex.argtypes = [sk, vp, ctypes.c_int, ctypes.c_int, i64, vp, ctypes.c_int,
                               ctypes.c_int, i64, i64, i64, i64, vp, ctypes.c_int, ctypes.c_int,
                               vp, i64, vp, sz, vp]
    gp = ctypes.POINTER(_GramProblem)
    L.os_gram_plan_create.restype = ctypes.c_int
    L.os_gram_plan_create.argtypes = [gp, i32, ctypes.c_int, ctypes.POINTER(vp)]
    L.os_gram_plan_destroy.restype = None
    L.os_gram_plan_destroy.argtypes = [vp]
    L.os_gram_workspace_bytes.restype = sz
    L.os_gram_workspace_bytes.argtypes = [vp]
    L.os_gram_configure.restype = ctypes.c_int
    L.os_gram_configure.argtypes = [vp, i32, i32, vp, sz, vp]
    L.os_gram_config.restype = None
    L.os_gram_config.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.os_gram_run.restype = ctypes.c_int
    L.os_gram_run.argtypes = [vp, ctypes.c_int, vp, sz, vp]
    L.os_gram_autotune.restype = ctypes.c_int
    L.os_gram_autotune.argtypes = [vp, i32, vp, sz, vp, ctypes.POINTER(ctypes.c_float)]
    L.os_gram_autotune_ex.restype = ctypes.c_int
    L.os_gram_autotune_ex.argtypes = [vp, i32, vp, sz, vp, ctypes.POINTER(_GramCandidate), i32,
                                      ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    L.os_gram_graph_create.restype = ctypes.c_int
    L.os_gram_graph_create.argtypes = [vp, ctypes.c_int, vp, sz, vp, ctypes.POINTER(vp)]
    L.os_graph_launch.restype = ctypes.c_int
    L.os_graph_launch.argtypes = [vp, vp]
    L.os_graph_destroy.restype = None
    L.os_graph_destroy.argtypes = [vp]
    _lib = L
    return L


def _check(status: int, what: str):
    if status != OS_OK:
        L = lib()
        msg = L.os_status_string(status).decode()
        if status == -5:
            msg += " (hipError_t %d)" % L.os_last_hip_error()
        raise OversketchError("%s: %s" % (what, msg), status)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _empty(shape, dtype, device, stream=None):
    """torch.empty on the caller's device.  The caching allocator ties a
    block to the stream that was current when it was allocated; when the
    kernels run on another (explicit) stream, the tensor is also recorded on
    that stream, so a temporary dropped on return is not handed to another
    allocation while the kernels still use it."""
    torch = _torch()
    t = torch.empty(shape, dtype=dtype, device=device)
    if stream is not None and stream != torch.cuda.current_stream(t.device):
        t.record_stream(stream)
    return t


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require_cuda(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise OversketchError("%s must be a CUDA (HIP) tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise OversketchError("%s must be %s, got %s" % (name, dtype, t.dtype))


def _row_major(t, name):
    """(rows, cols, ld) of a 2-D tensor with unit column stride."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise OversketchError("%s must be 2-D with unit column stride" % name)
    rows, cols = t.shape
    # a single row never uses its leading dimension: report its stride when
    # that is a valid one, else an aligned one
    if rows > 1 or t.stride(0) >= cols:
        return rows, cols, t.stride(0)
    return rows, cols, (cols + 15) // 16 * 16


def _sketch(b, N, e, seed, h=None, sigma=None, n=None):
    """The os_sketch struct.  Explicit tables must be [N+e, n] (the kernels
    read h[i*n + k]); n is required with them, so a table of the wrong width
    is refused here, before any launch."""
    s = _Sketch()
    s.seed = int(seed) & (2**64 - 1)
    s.b, s.N, s.e = int(b), int(N), int(e)
    s.h = None
    s.sigma = None
    if (h is None) != (sigma is None):
        raise OversketchError("explicit h and sigma go together")
    if h is not None:
        torch = _torch()
        if n is None:
            raise OversketchError("explicit h and sigma need the sketched length n")
        want = (int(N) + int(e), int(n))
        for t, name in ((h, "h"), (sigma, "sigma")):
            if not isinstance(t, torch.Tensor) or tuple(t.shape) != want:
                raise OversketchError("%s must be an [N+e, n] = [%d, %d] tensor, got %s"
                                      % (name, want[0], want[1],
                                         tuple(getattr(t, "shape", ()))))
        _require_cuda(h, "h", torch.int32)
        _require_cuda(sigma, "sigma", torch.int8)
        if not (h.is_contiguous() and sigma.is_contiguous()):
            raise OversketchError("h and sigma must be contiguous")
        s.h = h.data_ptr()
        s.sigma = sigma.data_ptr()
    return s


def _mask(keep, count):
    if keep is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(keep, dtype=np.uint8).reshape(-1))
    if arr.size != count:
        raise OversketchError("keep mask needs %d entries, got %d" % (count, arr.size))
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def block_stride(b: int) -> int:
    """Columns taken by one stored block (b rounded up to a multiple of 32)."""
    return int(lib().os_block_stride(int(b)))


def stored_count(N: int, e: int, keep=None, kept_only: bool = False) -> int:
    """Blocks a sketch stores: N+e, or the number kept when kept_only."""
    if not kept_only:
        return N + e
    if keep is None:
        return N
    return int(np.count_nonzero(np.asarray(keep)))


def hash_fill(n, b, N, e, seed=0, h=None, sigma=None, device="cuda", stream=None):
    """Buckets (int32) and signs (int8), each [N+e, n], computed on the GPU."""
    torch = _torch()
    s = _sketch(b, N, e, seed, h, sigma, n)
    h_out = _empty((N + e, n), torch.int32, device, stream)
    s_out = _empty((N + e, n), torch.int8, device, stream)
    _check(lib().os_hash_fill(ctypes.byref(s), n, _ptr(h_out), _ptr(s_out), _stream(stream)),
           "os_hash_fill")
    return h_out, s_out


OS_PREPARE_GROUPED = 1


def sketch_prepare(n, b, N, e, seed=0, h=None, sigma=None, device="cuda", stream=None,
                   grouped=False):
    """Prepared sketch (opaque uint8 device buffer) for an n-long sketched
    dimension.  grouped=True: buckets of similar list lengths share the
    sketch kernel's 64-bucket groups (fewer padding entries); the sketch's
    columns then hold each block's buckets in bucket_order.  The whole-path
    calls prepare in the natural order."""
    torch = _torch()
    s = _sketch(b, N, e, seed, h, sigma, n)
    nbytes = int(lib().os_sketch_prepare_bytes(ctypes.byref(s), n))
    if nbytes == 0:
        raise OversketchError("invalid sketch parameters")
    prep = _empty(nbytes, torch.uint8, device, stream)
    flags = OS_PREPARE_GROUPED if grouped else 0
    _check(lib().os_sketch_prepare_ex(ctypes.byref(s), n, flags, _ptr(prep), nbytes,
                                      _stream(stream)), "os_sketch_prepare_ex")
    return prep


def list_entries(prep, n, b, N, e, seed=0, h=None, sigma=None, stream=None):
    """(walked, real): list entries the sketch kernel walks per 4 lines,
    padding included, and the real ones (synchronous)."""
    s = _sketch(b, N, e, seed, h, sigma, n)
    w, r = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().os_sketch_list_entries(ctypes.byref(s), n, _ptr(prep), prep.numel(),
                                        ctypes.byref(w), ctypes.byref(r), _stream(stream)),
           "os_sketch_list_entries")
    return int(w.value), int(r.value)


def bucket_order(prep, n, b, N, e, seed=0, h=None, sigma=None, stream=None):
    """int32 [N+e, block_stride(b)]: the bucket held at each column of each
    block of a sketch taken with `prep` (the identity unless grouped)."""
    torch = _torch()
    s = _sketch(b, N, e, seed, h, sigma, n)
    order = _empty((N + e, block_stride(b)), torch.int32, prep.device, stream)
    _check(lib().os_sketch_bucket_order(ctypes.byref(s), n, _ptr(prep), prep.numel(),
                                        _ptr(order), _stream(stream)), "os_sketch_bucket_order")
    return order


def _line_major_out(out, lines, width, device, stream=None):
    torch = _torch()
    if out is None:
        return _empty((lines, width), torch.float32, device, stream)
    _require_cuda(out, "out", torch.float32)
    if tuple(out.shape) != (lines, width):
        raise OversketchError("out must be %d x %d" % (lines, width))
    return out


def sketch_cols(X, b, N, e, seed=0, keep=None, kept_only=False, h=None, sigma=None, prep=None,
                out=None, stream=None):
    """Line-major X S_i for the stored blocks, side by side: rows x (nst * block_stride(b))."""
    torch = _torch()
    _require_cuda(X, "X", torch.float32)
    rows, n, ldx = _row_major(X, "X")
    if prep is None:
        prep = sketch_prepare(n, b, N, e, seed, h, sigma, device=X.device, stream=stream)
    s = _sketch(b, N, e, seed, h, sigma, n)
    width = stored_count(N, e, keep, kept_only) * block_stride(b)
    out = _line_major_out(out, rows, width, X.device, stream)
    _, _, ldo = _row_major(out, "out")
    _, pk = _mask(keep, N + e)
    _check(lib().os_sketch_cols(ctypes.byref(s), _ptr(prep), prep.numel(), _ptr(X), rows, n, ldx,
                                pk, int(bool(kept_only)), _ptr(out), ldo, _stream(stream)),
           "os_sketch_cols")
    return out


def sketch_rows_workspace_bytes(n, cols) -> int:
    """Device workspace bytes of the transposing sketch_rows path."""
    return int(lib().os_sketch_rows_workspace_bytes(n, cols))


def sketch_rows(X, b, N, e, seed=0, keep=None, kept_only=False, h=None, sigma=None, prep=None,
                out=None, workspace=None, stream=None):
    """Line-major (S_i^T X)^T for the stored blocks, side by side: cols x (nst * block_stride(b)).

    workspace: None (sketch X's columns in place), True (allocate one) or a
    uint8 CUDA tensor of at least sketch_rows_workspace_bytes(n, cols) bytes
    (X is transposed into it first: the faster path).  X may be float32 or
    bfloat16; a bfloat16 X always takes the transposing path (converted
    exactly to FP32, FP32 sums)."""
    torch = _torch()
    _require_cuda(X, "X")
    if X.dtype not in (torch.float32, torch.bfloat16):
        raise OversketchError("X must be float32 or bfloat16")
    n, cols, ldx = _row_major(X, "X")
    if prep is None:
        prep = sketch_prepare(n, b, N, e, seed, h, sigma, device=X.device, stream=stream)
    s = _sketch(b, N, e, seed, h, sigma, n)
    width = stored_count(N, e, keep, kept_only) * block_stride(b)
    out = _line_major_out(out, cols, width, X.device, stream)
    _, _, ldo = _row_major(out, "out")
    _, pk = _mask(keep, N + e)
    if workspace is True or (workspace is None and X.dtype == torch.bfloat16):
        workspace = _empty(sketch_rows_workspace_bytes(n, cols), torch.uint8, X.device, stream)
    wp, wn = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel())
    dtype = 1 if X.dtype == torch.bfloat16 else 0
    _check(lib().os_sketch_rows_ex(ctypes.byref(s), _ptr(prep), prep.numel(), _ptr(X), dtype, n,
                                   cols, ldx, pk, int(bool(kept_only)), _ptr(out), ldo, wp, wn,
                                   _stream(stream)),
           "os_sketch_rows_ex")
    return out


def gemm_kept(At, Bt, b, keep=None, out=None, stream=None):
    """(1/K) sum over kept stored blocks j of At_j Bt_j^T (m x l), At and Bt
    line-major sketches (m x (nst * block_stride(b)) and l x (nst * block_stride(b)))."""
    torch = _torch()
    _require_cuda(At, "At", torch.float32)
    _require_cuda(Bt, "Bt", torch.float32)
    m, wa, lda = _row_major(At, "At")
    l, wb, ldb = _row_major(Bt, "Bt")
    bp = block_stride(b)
    if wa != wb or wa % bp:
        raise OversketchError("At and Bt must both hold nst * block_stride(b) columns")
    nst = wa // bp
    if out is None:
        out = _empty((m, l), torch.float32, At.device, stream)
    _require_cuda(out, "out", torch.float32)
    _, _, ldc = _row_major(out, "out")
    _, pk = _mask(keep, nst)
    _check(lib().os_gemm_kept(_ptr(At), lda, _ptr(Bt), ldb, m, l, int(b), nst, pk, _ptr(out), ldc,
                              _stream(stream)), "os_gemm_kept")
    return out


def _prec(precision) -> int:
    if precision not in PRECISIONS:
        raise OversketchError("precision must be one of %s" % sorted(PRECISIONS))
    return PRECISIONS[precision]


def block_stride_prec(b: int, precision: str = "fp32") -> int:
    """Columns taken by one stored block in a sketch of the given precision."""
    return int(lib().os_block_stride_prec(int(b), _prec(precision)))


def quantized_row(b, nst, precision) -> int:
    """Length of a row of a quantized sketch: BF16 values, or bytes for the
    FP8 forms (codes, then one scale byte per 64 codes)."""
    return int(lib().os_quantized_row(int(b), int(nst), _prec(precision)))


def sketch_quantize(S, b, nst, precision="bf16", out=None, stream=None):
    """Low-precision copy of a line-major FP32 sketch (lines x nst*block_stride(b))
    for gemm_kept_prec: BF16 (lines x quantized_row) or, for the FP8 forms,
    uint8 (lines x quantized_row bytes: E4M3 codes, then the E8M0 scales)."""
    torch = _torch()
    _require_cuda(S, "S", torch.float32)
    lines, _, lds = _row_major(S, "S")
    p = _prec(precision)
    width = quantized_row(b, nst, precision)
    fp8 = precision.startswith("fp8")
    dt = torch.uint8 if fp8 else torch.bfloat16
    pad = 16 if fp8 else 8                      # rows of 16 bytes
    if out is None:
        out = _empty((lines, (width + pad - 1) // pad * pad), dt, S.device, stream)[:, :width]
    _require_cuda(out, "out", dt)
    _, w, ldq = _row_major(out, "out")
    if w != width:
        raise OversketchError("out must have %d columns" % width)
    _check(lib().os_sketch_quantize(_ptr(S), lines, lds, int(b), int(nst), p, _ptr(out), ldq,
                                    _stream(stream)), "os_sketch_quantize")
    return out


def gemm_kept_prec(At, Bt, b, nst, precision="bf16", keep=None, out=None, stream=None):
    """Block product over the kept stored blocks with BF16 operands from
    sketch_quantize (FP32 accumulation); "fp32" takes FP32 sketches as
    gemm_kept does."""
    torch = _torch()
    p = _prec(precision)
    dt = {"fp32": torch.float32, "bf16": torch.bfloat16, "bf16x3": torch.bfloat16,
          "fp8": torch.uint8, "fp8x3": torch.uint8}[precision]
    _require_cuda(At, "At", dt)
    _require_cuda(Bt, "Bt", dt)
    m, _, lda = _row_major(At, "At")
    l, _, ldb = _row_major(Bt, "Bt")
    if out is None:
        out = _empty((m, l), torch.float32, At.device, stream)
    _require_cuda(out, "out", torch.float32)
    _, _, ldc = _row_major(out, "out")
    _, pk = _mask(keep, nst)
    _check(lib().os_gemm_kept_prec(_ptr(At), lda, _ptr(Bt), ldb, m, l, int(b), int(nst), pk, p,
                                   _ptr(out), ldc, _stream(stream)), "os_gemm_kept_prec")
    return out


def workspace_bytes(m, n, l, b, N, e, b_col_major=False, precision="fp32") -> int:
    """Device workspace bytes of matmul (B row-major unless b_col_major)."""
    s = _sketch(b, N, e, 0)
    return int(lib().os_matmul_prec_workspace_bytes(ctypes.byref(s), m, n, l,
                                                    int(bool(b_col_major)), _prec(precision)))


def matmul(A, B, b, N, e, seed=0, keep=None, kept_only=False, h=None, sigma=None, out=None,
           workspace=None, stream=None, precision="fp32"):
    """OverSketch product C ~= (1/K) sum_{kept i} (A S_i)(S_i^T B).

    A: m x n float32 with unit column stride.  B: n x l float32, either with
    unit column stride (row-major) or unit row stride (column-major, e.g. the
    transpose of a contiguous l x n tensor).  keep: host mask over the N+e
    blocks (None = the first N).  precision: operands of the block product,
    "fp32", "bf16" or "bf16x3" (split BF16); FP32 accumulation.  workspace:
    optional uint8 CUDA tensor of at least workspace_bytes(...) bytes.
    """
    torch = _torch()
    _require_cuda(A, "A", torch.float32)
    _require_cuda(B, "B", torch.float32)
    m, n, lda = _row_major(A, "A")
    if B.dim() != 2 or B.shape[0] != n:
        raise OversketchError("B must be n x l")
    l = B.shape[1]
    if B.stride(1) == 1 and (B.stride(0) != 1 or l == 1 and n > 1):
        b_col_major, ldb = 0, B.stride(0) if n > 1 else (l + 3) // 4 * 4
    elif B.stride(0) == 1:
        b_col_major, ldb = 1, B.stride(1) if l > 1 else (n + 3) // 4 * 4
    else:
        raise OversketchError("B must have a unit stride in one dimension")
    p = _prec(precision)
    s = _sketch(b, N, e, seed, h, sigma, n)
    need = int(lib().os_matmul_prec_workspace_bytes(ctypes.byref(s), m, n, l, b_col_major, p))
    if need == 0:
        raise OversketchError("invalid sizes for os_matmul")
    if workspace is None:
        workspace = _empty(need, torch.uint8, A.device, stream)
    if out is None:
        out = _empty((m, l), torch.float32, A.device, stream)
    _require_cuda(out, "out", torch.float32)
    _, _, ldc = _row_major(out, "out")
    _, pk = _mask(keep, N + e)
    _check(lib().os_matmul_prec(ctypes.byref(s), _ptr(A), lda, _ptr(B), ldb, b_col_major, m, n,
                                l, pk, int(bool(kept_only)), p, _ptr(out), ldc, _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream)),
           "os_matmul_prec")
    return out


def noalloc_scratch_bytes() -> int:
    """Bytes of the library's fixed device scratch (os_matmul_noalloc)."""
    return int(lib().os_noalloc_scratch_bytes())


def matmul_noalloc(A, B, b, N, e, out, seed=0, keep=None, kept_only=False, h=None, sigma=None,
                   stream=None, precision="fp32"):
    """matmul with the library's fixed scratch as workspace (os_matmul_noalloc):
    nothing is allocated, so `out` (m x l float32) is required.  Calls that
    overlap on one GPU race on the shared scratch."""
    torch = _torch()
    _require_cuda(A, "A", torch.float32)
    _require_cuda(B, "B", torch.float32)
    _require_cuda(out, "out", torch.float32)
    m, n, lda = _row_major(A, "A")
    if B.dim() != 2 or B.shape[0] != n:
        raise OversketchError("B must be n x l")
    l = B.shape[1]
    if B.stride(1) == 1 and (B.stride(0) != 1 or l == 1 and n > 1):
        b_col_major, ldb = 0, B.stride(0) if n > 1 else (l + 3) // 4 * 4
    elif B.stride(0) == 1:
        b_col_major, ldb = 1, B.stride(1) if l > 1 else (n + 3) // 4 * 4
    else:
        raise OversketchError("B must have a unit stride in one dimension")
    if tuple(out.shape) != (m, l):
        raise OversketchError("out must be %d x %d" % (m, l))
    _, _, ldc = _row_major(out, "out")
    s = _sketch(b, N, e, seed, h, sigma, n)
    _, pk = _mask(keep, N + e)
    _check(lib().os_matmul_noalloc(ctypes.byref(s), _ptr(A), lda, _ptr(B), ldb, b_col_major, m, n,
                                   l, pk, int(bool(kept_only)), _prec(precision), _ptr(out), ldc,
                                   _stream(stream)), "os_matmul_noalloc")
    return out


def _cmask_tensor(cmask, nbI, nbJ, nst, device, stream=None):
    torch = _torch()
    if not isinstance(cmask, torch.Tensor):
        cmask = torch.from_numpy(np.ascontiguousarray(np.asarray(cmask, dtype=np.uint8)))
    cmask = cmask.to(device=device, dtype=torch.uint8).contiguous()
    if tuple(cmask.shape) != (nbI, nbJ, nst):
        raise OversketchError("cmask must be %d x %d x %d" % (nbI, nbJ, nst))
    cur = torch.cuda.current_stream(cmask.device)
    if stream is not None and stream != cur:
        # the copy above ran on the current stream: the kernels' stream waits for it
        stream.wait_stream(cur)
        cmask.record_stream(stream)
    return cmask


def gemm_kept_cmask(At, Bt, b, cmask, out=None, stream=None):
    """Block product with a keep mask per b x b block of C: cmask
    [ceil(m/b), ceil(l/b), nst] (host array or CUDA tensor)."""
    torch = _torch()
    _require_cuda(At, "At", torch.float32)
    _require_cuda(Bt, "Bt", torch.float32)
    m, wa, lda = _row_major(At, "At")
    l, wb, ldb = _row_major(Bt, "Bt")
    bp = block_stride(b)
    if wa != wb or wa % bp:
        raise OversketchError("At and Bt must both hold nst * block_stride(b) columns")
    nst = wa // bp
    cm = _cmask_tensor(cmask, -(-m // b), -(-l // b), nst, At.device, stream)
    if out is None:
        out = _empty((m, l), torch.float32, At.device, stream)
    _require_cuda(out, "out", torch.float32)
    _, _, ldc = _row_major(out, "out")
    _check(lib().os_gemm_kept_cmask(_ptr(At), lda, _ptr(Bt), ldb, m, l, int(b), nst, _ptr(cm),
                                    _ptr(out), ldc, _stream(stream)), "os_gemm_kept_cmask")
    return out


def matmul_cmask(A, B, b, N, e, cmask, seed=0, h=None, sigma=None, out=None, workspace=None,
                 stream=None):
    """OverSketch product with a keep mask per b x b block of C: cmask
    [ceil(m/b), ceil(l/b), N+e]; every block is sketched."""
    torch = _torch()
    _require_cuda(A, "A", torch.float32)
    _require_cuda(B, "B", torch.float32)
    m, n, lda = _row_major(A, "A")
    if B.dim() != 2 or B.shape[0] != n:
        raise OversketchError("B must be n x l")
    l = B.shape[1]
    if B.stride(1) == 1 and (B.stride(0) != 1 or l == 1 and n > 1):
        b_col_major, ldb = 0, B.stride(0) if n > 1 else (l + 3) // 4 * 4
    elif B.stride(0) == 1:
        b_col_major, ldb = 1, B.stride(1) if l > 1 else (n + 3) // 4 * 4
    else:
        raise OversketchError("B must have a unit stride in one dimension")
    s = _sketch(b, N, e, seed, h, sigma, n)
    cm = _cmask_tensor(cmask, -(-m // b), -(-l // b), N + e, A.device, stream)
    need = int(lib().os_matmul_prec_workspace_bytes(ctypes.byref(s), m, n, l, b_col_major, 0))
    if need == 0:
        raise OversketchError("invalid sizes for os_matmul_cmask")
    if workspace is None:
        workspace = _empty(need, torch.uint8, A.device, stream)
    if out is None:
        out = _empty((m, l), torch.float32, A.device, stream)
    _require_cuda(out, "out", torch.float32)
    _, _, ldc = _row_major(out, "out")
    _check(lib().os_matmul_cmask(ctypes.byref(s), _ptr(A), lda, _ptr(B), ldb, b_col_major, m, n,
                                 l, _ptr(cm), _ptr(out), ldc, _ptr(workspace),
                                 workspace.numel() * workspace.element_size(), _stream(stream)),
           "os_matmul_cmask")
    return out


def _layout(t, name):
    """(dtype code, col_major, rows, cols, ld) of a 2-D float32 / bfloat16
    tensor with unit stride along one of its dimensions."""
    torch = _torch()
    _require_cuda(t, name)
    if t.dtype == torch.float32:
        code = 0
    elif t.dtype == torch.bfloat16:
        code = 1
    else:
        raise OversketchError("%s must be float32 or bfloat16" % name)
    if t.dim() != 2:
        raise OversketchError("%s must be 2-D" % name)
    rows, cols = t.shape
    if t.stride(1) == 1 and (rows == 1 or t.stride(0) >= cols):
        return code, 0, rows, cols, t.stride(0) if rows > 1 else max(cols, 1)
    if t.stride(0) == 1 and (cols == 1 or t.stride(1) >= rows):
        return code, 1, rows, cols, t.stride(1) if cols > 1 else max(rows, 1)
    raise OversketchError("%s must have unit stride along one dimension" % name)


def matmul_ex(A, B, b, N, e, seed=0, keep=None, kept_only=False, precision="fp32", h=None,
              sigma=None, out=None, workspace=None, stream=None):
    """os_matmul_ex: C ~= A S S^T B for A (m x n) and B (n x l) given as
    float32 or bfloat16 tensors, row- or column-major (a transposed view is
    column-major), in either type and layout.
    Returns C (m x l, float32)."""
    torch = _torch()
    ad, acm, m, n, lda = _layout(A, "A")
    bd, bcm, n2, l, ldb = _layout(B, "B")
    if n2 != n:
        raise OversketchError("inner dimensions differ")
    sk = _sketch(b, N, e, seed, h, sigma, n)
    arr, kp = _mask(keep, int(N) + int(e))
    prec = _prec(precision)
    L = lib()
    need = int(L.os_matmul_ex_workspace_bytes(ctypes.byref(sk), m, n, l, acm, bcm, prec))
    if need == 0:
        raise OversketchError("invalid sizes or sketch parameters")
    if workspace is None or workspace.numel() < need:
        workspace = _empty(need, torch.uint8, A.device, stream)
    if out is None:
        out = _empty((m, l), torch.float32, A.device, stream)
    _, _, ldc = _row_major(out, "out")
    _check(L.os_matmul_ex(ctypes.byref(sk), _ptr(A), ad, acm, lda, _ptr(B), bd, bcm, ldb, m, n, l,
                          kp, 1 if kept_only else 0, prec, _ptr(out), ldc, _ptr(workspace),
                          workspace.numel(), _stream(stream)), "os_matmul_ex")
    return out


from .gram import GramBatch  # noqa: E402  (uses the helpers above)
