"""The C-ABI library: it loads, exports every entry point the header declares,
and rejects invalid arguments before touching the GPU (host-only checks; no
compute call is made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1811_02653_amd as osk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oversketch.h")

OS_OK, OS_EINVAL, OS_ENULL, OS_EALIGN, OS_EWORKSPACE, OS_EHIP, OS_ENOKEEP = 0, -1, -2, -3, -4, -5, -6

# A fake, 256-byte-aligned "device" address: validation never dereferences it
# and every call below fails validation before any launch.
FAKE = ctypes.c_void_p(1 << 20)


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?(os_[a-z_]+)\(", text, re.M)))


def _sk(b=64, N=4, e=1, seed=1):
    s = osk._Sketch()
    s.seed, s.b, s.N, s.e, s.h, s.sigma = seed, b, N, e, None, None
    return s


@pytest.fixture(scope="module")
def L():
    return osk.lib()


def test_header_declares_the_path(L):
    names = _declared()
    for want in ["os_hash_fill", "os_sketch_prepare_bytes", "os_sketch_prepare", "os_sketch_cols",
                 "os_sketch_rows", "os_sketch_rows_workspace_bytes", "os_gemm_kept", "os_matmul",
                 "os_matmul_workspace_bytes",
                 "os_status_string", "os_last_hip_error", "os_block_stride"]:
        assert want in names


def test_every_declared_symbol_is_exported(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings(L):
    for code in (OS_OK, OS_EINVAL, OS_ENULL, OS_EALIGN, OS_EWORKSPACE, OS_EHIP, OS_ENOKEEP):
        assert L.os_status_string(code)
    assert L.os_status_string(123) == b"unknown os_status"
    assert L.os_last_hip_error() == 0


def test_block_stride(L):
    assert [L.os_block_stride(b) for b in (0, 1, 31, 32, 33, 256, 1000, 1024)] == \
        [0, 32, 32, 32, 64, 256, 1024, 1024]


def test_prepare_and_workspace_bytes(L):
    s = _sk(b=1000, N=8, e=2)
    n = 32769
    prep = L.os_sketch_prepare_bytes(ctypes.byref(s), n)
    r256 = lambda x: (x + 255) // 256 * 256
    table = 10 * 32772 * 4
    nwin, qn = 5, 16                          # windows of 8192 indices, groups of 64 buckets
    rc = 8192 // 8 + qn                       # 1 KiB chunks per (block, window)
    lists = r256(10 * nwin * qn * 4) + 10 * nwin * rc * 1024
    inv = r256(10 * 1024 * 4)                 # bucket -> column map per block (bp = 1024)
    assert prep == r256(table) + r256(lists) + inv
    small = L.os_sketch_prepare_bytes(ctypes.byref(_sk(b=64, N=1, e=0)), 100)
    assert small == (r256(1 * 100 * 4) + r256(r256(1 * 1 * 1 * 4) + 1 * 1 * ((100 + 7) // 8 + 1)
                                               * 1024) + r256(64 * 4))
    m, l = 300, 77
    ws = L.os_matmul_workspace_bytes(ctypes.byref(s), m, n, l, 1)      # column-major B
    # the FP32 product's split K loop: 2 tiles of 256 x 256, at most 10 * 1024 / 32
    # K steps, so min(256 / 2, 320 / 2) = 128 partial products of 300 x 77
    split = r256(128 * 300 * 77 * 4)
    assert ws == r256(prep) + r256(300 * 10 * 1024 * 4) + r256(77 * 10 * 1024 * 4) + split
    # no split with enough tiles to fill the device (16 x 16 tiles)
    big = L.os_matmul_workspace_bytes(ctypes.byref(s), 4096, n, 4096, 1)
    assert big == r256(prep) + r256(4096 * 10 * 1024 * 4) * 2
    # BF16 operands: the BF16 copies (10 blocks of 1024 values per row) and a split
    # area for at most 10 * 1024 / 64 = 160 K steps: min(128, 80) partial products
    bf = L.os_matmul_prec_workspace_bytes(ctypes.byref(s), m, n, l, 1, 1)
    assert bf == (r256(prep) + r256(300 * 10 * 1024 * 4) + r256(77 * 10 * 1024 * 4) +
                  r256(300 * 10 * 1024 * 2) + r256(77 * 10 * 1024 * 2) +
                  r256(80 * 300 * 77 * 4))
    transposed = r256(77 * 32772 * 4)                                   # B^T, ld n rounded to 4
    assert L.os_matmul_workspace_bytes(ctypes.byref(s), m, n, l, 0) == ws + transposed
    assert L.os_sketch_rows_workspace_bytes(n, l) == transposed
    assert L.os_sketch_rows_workspace_bytes(0, l) == 0
    bad = _sk(b=0)
    assert L.os_sketch_prepare_bytes(ctypes.byref(bad), 10) == 0
    assert L.os_matmul_workspace_bytes(ctypes.byref(bad), 1, 1, 1, 0) == 0
    assert L.os_sketch_prepare_bytes(ctypes.byref(s), 0) == 0


@pytest.mark.parametrize("b,N,e", [(0, 1, 0), (8193, 1, 0), (4, 0, 1), (4, 2, -1), (4, 200, 57)])
def test_sketch_parameters_rejected(L, b, N, e):
    s = _sk(b=b, N=N, e=e)
    assert L.os_sketch_prepare(ctypes.byref(s), 10, FAKE, 1 << 30, None) == OS_EINVAL
    assert L.os_matmul(ctypes.byref(s), FAKE, 16, FAKE, 16, 0, 4, 16, 4, None, 0, FAKE, 4, FAKE,
                       1 << 30, None) == OS_EINVAL


BIG = 1 << 30   # a prepared-buffer size that always suffices here


def test_null_and_half_explicit_tables(L):
    assert L.os_sketch_prepare(None, 10, FAKE, BIG, None) == OS_ENULL
    s = _sk()
    s.h = 1 << 20          # explicit buckets without signs
    assert L.os_hash_fill(ctypes.byref(s), 10, FAKE, FAKE, None) == OS_ENULL
    s = _sk()
    assert L.os_hash_fill(ctypes.byref(s), 10, None, FAKE, None) == OS_ENULL
    assert L.os_sketch_cols(ctypes.byref(s), None, BIG, FAKE, 4, 16, 16, None, 0, FAKE, 320,
                            None) == OS_ENULL
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, None, 4, 16, 16, None, 0, FAKE, 320,
                            None) == OS_ENULL


def test_sizes_rejected(L):
    s = _sk()              # b = 64, N + e = 5: a sketch is 5 * 64 = 320 columns wide
    assert L.os_hash_fill(ctypes.byref(s), 0, FAKE, FAKE, None) == OS_EINVAL
    assert L.os_hash_fill(ctypes.byref(s), 1 << 31, FAKE, FAKE, None) == OS_EINVAL
    # lda < n
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, FAKE, 4, 16, 12, None, 0, FAKE, 320,
                            None) == OS_EINVAL
    # output ld < sketch width
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, FAKE, 8, 16, 16, None, 0, FAKE, 316,
                            None) == OS_EINVAL
    assert L.os_sketch_rows(ctypes.byref(s), FAKE, BIG, FAKE, 16, 8, 8, None, 0, FAKE, 316,
                            None, 0, None) == OS_EINVAL
    # transpose workspace too small or misaligned
    wneed = L.os_sketch_rows_workspace_bytes(16, 8)
    assert L.os_sketch_rows(ctypes.byref(s), FAKE, BIG, FAKE, 16, 8, 8, None, 0, FAKE, 320,
                            FAKE, wneed - 1, None) == OS_EWORKSPACE
    assert L.os_sketch_rows(ctypes.byref(s), FAKE, BIG, FAKE, 16, 8, 8, None, 0, FAKE, 320,
                            ctypes.c_void_p((1 << 20) + 16), wneed, None) == OS_EWORKSPACE
    # rows beyond the limit
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, FAKE, (1 << 24) + 1, 16, 16, None, 0, FAKE,
                            320, None) == OS_EINVAL
    # prepared buffer too small
    need = L.os_sketch_prepare_bytes(ctypes.byref(s), 16)
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, need - 1, FAKE, 4, 16, 16, None, 0, FAKE, 320,
                            None) == OS_EWORKSPACE
    assert L.os_sketch_prepare(ctypes.byref(s), 16, FAKE, need - 1, None) == OS_EWORKSPACE
    # gemm operands narrower than nst * bp
    assert L.os_gemm_kept(FAKE, 60, FAKE, 64, 4, 4, 64, 1, None, FAKE, 4, None) == OS_EINVAL
    # ldc < l
    assert L.os_matmul(ctypes.byref(s), FAKE, 16, FAKE, 8, 0, 4, 16, 8, None, 0, FAKE, 7, FAKE,
                       1 << 30, None) == OS_EINVAL


def test_alignment_rejected(L):
    s = _sk()
    odd = ctypes.c_void_p((1 << 20) + 4)
    assert L.os_sketch_prepare(ctypes.byref(s), 10, ctypes.c_void_p((1 << 20) + 16), BIG,
                               None) == OS_EALIGN
    # inputs need only 4-byte alignment: the failures below are the outputs'
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, odd, 4, 15, 15, None, 0, odd, 320,
                            None) == OS_EALIGN
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, odd, 4, 15, 15, None, 0, FAKE, 322,
                            None) == OS_EALIGN
    assert L.os_sketch_rows(ctypes.byref(s), FAKE, BIG, odd, 16, 4, 5, None, 0, FAKE, 321,
                            None, 0, None) == OS_EALIGN
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, ctypes.c_void_p((1 << 20) + 2), 4, 16, 16,
                            None, 0, FAKE, 320, None) == OS_EALIGN
    # sketches are read 16 bytes at a time by the product
    assert L.os_gemm_kept(odd, 64, FAKE, 64, 4, 4, 64, 1, None, FAKE, 4, None) == OS_EALIGN
    assert L.os_gemm_kept(FAKE, 66, FAKE, 64, 4, 4, 64, 1, None, FAKE, 4, None) == OS_EALIGN
    assert L.os_gemm_kept(FAKE, 64, FAKE, 64, 4, 4, 64, 1, None, ctypes.c_void_p((1 << 20) + 2), 4,
                          None) == OS_EALIGN


def test_keep_mask_rejected(L):
    s = _sk(N=2, e=1)
    none = np.zeros(3, dtype=np.uint8)
    p = none.ctypes.data_as(ctypes.c_void_p)
    assert L.os_sketch_cols(ctypes.byref(s), FAKE, BIG, FAKE, 4, 16, 16, p, 1, FAKE, 192,
                            None) == OS_ENOKEEP
    assert L.os_matmul(ctypes.byref(s), FAKE, 16, FAKE, 8, 0, 4, 16, 8, p, 0, FAKE, 8, FAKE,
                       1 << 30, None) == OS_ENOKEEP
    assert L.os_gemm_kept(FAKE, 192, FAKE, 192, 4, 4, 64, 3, p, FAKE, 4, None) == OS_ENOKEEP


def test_workspace_rejected(L):
    s = _sk()
    need = L.os_matmul_workspace_bytes(ctypes.byref(s), 4, 16, 8, 0)
    assert need > L.os_matmul_workspace_bytes(ctypes.byref(s), 4, 16, 8, 1) > 0
    assert L.os_matmul(ctypes.byref(s), FAKE, 16, FAKE, 8, 0, 4, 16, 8, None, 0, FAKE, 8, None,
                       need, None) == OS_EWORKSPACE
    assert L.os_matmul(ctypes.byref(s), FAKE, 16, FAKE, 8, 0, 4, 16, 8, None, 0, FAKE, 8, FAKE,
                       need - 1, None) == OS_EWORKSPACE
    assert L.os_matmul(ctypes.byref(s), FAKE, 16, FAKE, 8, 0, 4, 16, 8, None, 0, FAKE, 8,
                       ctypes.c_void_p((1 << 20) + 16), need, None) == OS_EWORKSPACE


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    A = torch.zeros(4, 16)
    with pytest.raises(osk.OversketchError):
        osk.matmul(A, torch.zeros(16, 4), b=4, N=2, e=0)


# ---------------------------------------------------------------------------
# batched Gram plans (host-only: plan creation validates without the GPU)
# ---------------------------------------------------------------------------

def _gram(m=300, n=6000, b=150, N=6, e=1, A=FAKE, d=None, keep=None, H=FAKE, lda=None, ldh=None):
    p = osk._GramProblem()
    p.sk = _sk(b=b, N=N, e=e)
    p.A, p.lda = A, (n if lda is None else lda)
    p.d = d
    p.m, p.n = m, n
    p.keep = keep
    p.H, p.ldh = H, (m if ldh is None else ldh)
    return p


def _create(L, probs, full=1):
    arr = (osk._GramProblem * max(len(probs), 1))(*probs)
    h = ctypes.c_void_p()
    st = L.os_gram_plan_create(arr, len(probs), full, ctypes.byref(h))
    return st, h


def test_gram_plan_rejects_bad_problems(L):
    none = np.zeros(7, dtype=np.uint8)
    cases = [
        ([], OS_EINVAL),
        ([_gram(b=0)], OS_EINVAL),
        ([_gram(m=0)], OS_EINVAL),
        ([_gram(A=None)], OS_ENULL),
        ([_gram(H=None)], OS_ENULL),
        ([_gram(A=ctypes.c_void_p((1 << 20) + 2))], OS_EALIGN),
        ([_gram(d=ctypes.c_void_p((1 << 20) + 1))], OS_EALIGN),
        ([_gram(lda=10)], OS_EINVAL),
        ([_gram(ldh=10)], OS_EINVAL),
        ([_gram(), _gram(keep=none.ctypes.data_as(ctypes.c_void_p))], OS_ENOKEEP),
    ]
    for probs, want in cases:
        st, h = _create(L, probs)
        assert st == want, (probs, st)
        assert not h.value
    h = ctypes.c_void_p(123)
    assert L.os_gram_plan_create(None, 1, 1, ctypes.byref(h)) == OS_ENULL and not h.value
    arr = (osk._GramProblem * 1)(_gram())
    assert L.os_gram_plan_create(arr, 1, 1, None) == OS_ENULL
    L.os_gram_plan_destroy(None)
    L.os_graph_destroy(None)
    assert L.os_graph_launch(None, None) == OS_ENULL


def test_gram_workspace_and_unconfigured_plan(L):
    st, h1 = _create(L, [_gram()])
    assert st == OS_OK and h1.value
    st, h2 = _create(L, [_gram(), _gram(m=1000, n=20000, b=500)])
    assert st == OS_OK
    w1, w2 = L.os_gram_workspace_bytes(h1), L.os_gram_workspace_bytes(h2)
    assert w1 % 256 == 0 and w2 % 256 == 0
    # at least the prepared sketch and the kept-block sketch (m x K*bp FP32)
    s = _sk(b=150, N=6, e=1)
    assert w1 >= L.os_sketch_prepare_bytes(ctypes.byref(s), 6000) + 300 * 6 * 160 * 4
    s2 = _sk(b=500, N=6, e=1)
    assert w2 - w1 >= L.os_sketch_prepare_bytes(ctypes.byref(s2), 20000) + 1000 * 6 * 512 * 4
    assert L.os_gram_workspace_bytes(None) == 0
    t, g = ctypes.c_int32(7), ctypes.c_int32(7)
    L.os_gram_config(h1, ctypes.byref(t), ctypes.byref(g))
    assert (t.value, g.value) == (0, 0)
    ws = ctypes.c_void_p(1 << 30)
    # not configured yet, or workspace too small / misaligned / NULL
    assert L.os_gram_run(h1, 7, ws, w1, None) == OS_EINVAL
    assert L.os_gram_run(h1, 7, ws, w1 - 1, None) == OS_EWORKSPACE
    assert L.os_gram_run(h1, 7, ctypes.c_void_p((1 << 30) + 64), w1, None) == OS_EALIGN
    assert L.os_gram_run(h1, 7, None, w1, None) == OS_ENULL
    assert L.os_gram_run(None, 7, ws, w1, None) == OS_ENULL
    assert L.os_gram_run(h1, 0, ws, w1, None) == OS_EINVAL        # no stage
    assert L.os_gram_run(h1, 8, ws, w1, None) == OS_EINVAL
    # bad tile or grid fails before any device query
    assert L.os_gram_configure(h1, 64, 0, ws, w1, None) == OS_EINVAL
    assert L.os_gram_configure(h1, 256, -1, ws, w1, None) == OS_EINVAL
    assert L.os_gram_configure(h1, 256, 1 << 20, ws, w1, None) == OS_EINVAL
    assert L.os_gram_configure(h1, 2, 0, ws, w1, None) == OS_EINVAL   # not a tile form
    assert L.os_gram_configure(h1, -1, 0, ws, w1, None) == OS_EINVAL
    assert L.os_gram_autotune(h1, 0, ws, w1, None, None) == OS_EINVAL
    n = ctypes.c_int32(9)
    assert L.os_gram_autotune_ex(h1, 0, ws, w1, None, None, 0, ctypes.byref(n), None) == OS_EINVAL
    assert n.value == 0
    assert L.os_gram_autotune_ex(h1, 1, ws, w1, None, None, -1, None, None) == OS_EINVAL
    assert L.os_gram_autotune_ex(h1, 1, ws, w1, None, None, 4, None, None) == OS_EINVAL
    assert L.os_gram_autotune_ex(None, 1, ws, w1, None, None, 0, None, None) == OS_ENULL
    assert L.os_gram_autotune_ex(h1, 1, ws, w1 - 1, None, None, 0, None, None) == OS_EWORKSPACE
    g = ctypes.c_void_p(5)
    assert L.os_gram_graph_create(h1, 7, ws, w1, ctypes.c_void_p(1), ctypes.byref(g)) == OS_EINVAL
    assert not g.value
    L.os_gram_plan_destroy(h1)
    L.os_gram_plan_destroy(h2)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU only: --gpus N > 1 exits with a message
    before it imports torch or touches a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("shape", [(5, 99), (5, 101), (4, 100), (6, 100), (500,)])
def test_explicit_tables_of_the_wrong_shape_are_refused(shape):
    """A table that is not [N+e, n] is refused in the binding, before any
    library call (the kernels read h[i*n + k]: a short row would run past
    the tensor, a long one would shift every later block)."""
    torch = pytest.importorskip("torch")
    h = torch.zeros(shape, dtype=torch.int32)
    s = torch.ones(shape, dtype=torch.int8)
    with pytest.raises(osk.OversketchError, match=r"\[N\+e, n\]"):
        osk._sketch(64, 4, 1, 0, h, s, n=100)
    # every wrapper that takes tables checks them before it launches
    with pytest.raises(osk.OversketchError, match=r"\[N\+e, n\]"):
        osk.hash_fill(100, 64, 4, 1, h=h, sigma=s, device="cpu")
    with pytest.raises(osk.OversketchError, match=r"\[N\+e, n\]"):
        osk.sketch_prepare(100, 64, 4, 1, h=h, sigma=s, device="cpu")


def test_explicit_tables_need_n_and_a_gpu():
    torch = pytest.importorskip("torch")
    h = torch.zeros((5, 100), dtype=torch.int32)
    s = torch.ones((5, 100), dtype=torch.int8)
    with pytest.raises(osk.OversketchError, match="sketched length n"):
        osk._sketch(64, 4, 1, 0, h, s)
    # the right shape on the host: refused as not a device tensor
    with pytest.raises(osk.OversketchError, match="CUDA"):
        osk._sketch(64, 4, 1, 0, h, s, n=100)
    with pytest.raises(osk.OversketchError, match="together"):
        osk._sketch(64, 4, 1, 0, h, None, n=100)


def test_fresh_sketch_keys_per_forward():
    """The linear layer's default draws a new 64-bit key per forward call
    (independent sketches across training steps), reproducibly under
    torch.manual_seed."""
    torch = pytest.importorskip("torch")
    from paper_1811_02653_amd.autograd import fresh_seed
    torch.manual_seed(3)
    keys = [fresh_seed() for _ in range(8)]
    assert len(set(keys)) == 8
    assert all(0 <= k < 2**64 for k in keys)
    assert any(k >= 2**32 for k in keys)
    torch.manual_seed(3)
    assert [fresh_seed() for _ in range(8)] == keys


def test_prepare_ex_flags_and_diagnostics_validate(L):
    s = _sk(b=256, N=4, e=1)
    need = L.os_sketch_prepare_bytes(ctypes.byref(s), 4096)
    assert L.os_sketch_prepare_ex(ctypes.byref(s), 4096, 2, FAKE, need, None) == OS_EINVAL
    assert L.os_sketch_prepare_ex(ctypes.byref(s), 4096, 1, FAKE, need - 1, None) == OS_EWORKSPACE
    assert L.os_sketch_prepare_ex(None, 4096, 1, FAKE, need, None) == OS_ENULL
    w, r = ctypes.c_int64(0), ctypes.c_int64(0)
    assert L.os_sketch_list_entries(ctypes.byref(s), 4096, FAKE, need, None, ctypes.byref(r),
                                    None) == OS_ENULL
    assert L.os_sketch_list_entries(ctypes.byref(s), 4096, FAKE, need - 1, ctypes.byref(w),
                                    ctypes.byref(r), None) == OS_EWORKSPACE
    assert L.os_sketch_bucket_order(ctypes.byref(s), 4096, FAKE, need, None, None) == OS_ENULL
    assert L.os_sketch_bucket_order(ctypes.byref(s), 0, FAKE, need, FAKE, None) == OS_EINVAL


def test_noalloc_rejects_oversized_problems_before_any_launch(L):
    # the workspace of the full-size product exceeds the fixed scratch: the
    # call returns OS_EWORKSPACE on the host (FAKE pointers are never used)
    s = _sk(b=1024, N=8, e=2)
    assert L.os_noalloc_scratch_bytes() == 256 << 20
    assert L.os_matmul_noalloc(ctypes.byref(s), FAKE, 32768, FAKE, 8192, 0, 8192, 32768, 8192,
                               None, 0, 0, FAKE, 8192, None) == OS_EWORKSPACE
    bad = _sk(b=0)
    assert L.os_matmul_noalloc(ctypes.byref(bad), FAKE, 16, FAKE, 16, 0, 4, 16, 4, None, 0, 0,
                               FAKE, 4, None) == OS_EINVAL
    assert L.os_matmul_noalloc(None, FAKE, 16, FAKE, 16, 0, 4, 16, 4, None, 0, 0, FAKE, 4,
                               None) == OS_ENULL
