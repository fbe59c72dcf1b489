"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs and the same sketch.

Tolerances (FP32 path against the FP64 oracle):
  - buckets and signs: bit-exact;
  - sketches of permutation / identity inputs (one term per bucket): bit-exact;
  - sketches of random inputs against the FP32 sum of each bucket taken term
    by term in ascending k (the order the bucket lists fix): bit-exact;
  - sketches of random inputs: relative Frobenius error <= 1e-6 per block
    (an FP32 sum of about n/b terms);
  - the product C: relative Frobenius error <= 1e-5.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1811_02653_amd as osk  # noqa: E402

SKETCH_TOL = 1e-6
PRODUCT_TOL = 1e-5


def dev(x, ld=None):
    """Host array -> CUDA float32 tensor view with leading dimension ld
    (rounded up to a multiple of 4 by default)."""
    x = np.asarray(x, dtype=np.float32)
    rows, cols = x.shape
    if ld is None:
        ld = (cols + 3) // 4 * 4
    buf = torch.zeros((rows, ld), dtype=torch.float32, device="cuda")
    buf[:, :cols] = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return buf[:, :cols]


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(x, y):
    return oracle.rel_frob(x, y)


def unpad(S, nst, b):
    """Line-major sketch (L x (nst * bp)) -> (L x nst*b) with the per-block
    padding columns dropped (they must be zero): the oracle's column layout."""
    bp = osk.block_stride(b)
    S = np.asarray(S)
    assert S.shape[1] == nst * bp
    for j in range(nst):
        assert np.all(S[:, j * bp + b:(j + 1) * bp] == 0), "padding columns must be zero"
    return np.concatenate([S[:, j * bp:j * bp + b] for j in range(nst)], axis=1)


def stored_blocks(N, e, keep, kept_only):
    if not kept_only:
        return list(range(N + e))
    if keep is None:
        return list(range(N))
    return [int(i) for i in np.flatnonzero(keep)]


# ---------------------------------------------------------------------------
# hash
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,b,N,e,n", [(0, 256, 4, 1, 4096), (12345, 1000, 8, 2, 1003),
                                          (2**63 + 7, 7, 1, 0, 5), (99, 1, 3, 3, 64)])
def test_hash_bit_exact(seed, b, N, e, n):
    h, s = osk.hash_fill(n, b, N, e, seed=seed)
    ho, so = oracle.hash_tables(seed, N + e, n, b)
    np.testing.assert_array_equal(h.cpu().numpy(), ho)
    np.testing.assert_array_equal(s.cpu().numpy(), so)


def test_prepared_sketch_is_reusable():
    # one prepared buffer serves both sketch kinds and any mask
    n, b, N, e, seed = 1001, 100, 3, 2, 5
    prep = osk.sketch_prepare(n, b, N, e, seed=seed)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((20, n)).astype(np.float32)
    keep = np.array([1, 0, 1, 1, 0], np.uint8)
    a = host(osk.sketch_cols(dev(X), b, N, e, seed=seed, prep=prep, keep=keep, kept_only=True))
    c = host(osk.sketch_cols(dev(X), b, N, e, seed=seed, keep=keep, kept_only=True))
    np.testing.assert_array_equal(a, c)
    h, s = oracle.hash_tables(seed, N + e, n, b)
    ref = oracle.sketch_cols(X, h, s, b)
    kept = [0, 2, 3]
    got = unpad(a, 3, b)
    for jj, i in enumerate(kept):
        assert rel(got[:, jj * b:(jj + 1) * b], ref[:, i * b:(i + 1) * b]) <= SKETCH_TOL


def test_explicit_tables_pass_through():
    n, b, N, e = 50, 8, 2, 1
    rng = np.random.default_rng(1)
    h = rng.integers(0, b, size=(N + e, n)).astype(np.int32)
    s = rng.choice(np.array([-1, 1], np.int8), size=(N + e, n))
    hd, sd = osk.hash_fill(n, b, N, e, h=torch.from_numpy(h).cuda(), sigma=torch.from_numpy(s).cuda())
    np.testing.assert_array_equal(hd.cpu().numpy(), h)
    np.testing.assert_array_equal(sd.cpu().numpy(), s)


# ---------------------------------------------------------------------------
# sketches
# ---------------------------------------------------------------------------

def test_paper_worked_example_on_gpu():
    # Section 4.1, Eq. (count_sketch_example): h (1-based) = 2 2 3 1 1 2 1 3 3,
    # signs + - + + - + - - -; sketching I_9 gives the printed S_c.
    h = np.array([[1, 1, 2, 0, 0, 1, 0, 2, 2]], dtype=np.int32)
    s = np.array([[1, -1, 1, 1, -1, 1, -1, -1, -1]], dtype=np.int8)
    ST = np.array([[0, 0, 0, 1, -1, 0, -1, 0, 0],
                   [1, -1, 0, 0, 0, 1, 0, 0, 0],
                   [0, 0, 1, 0, 0, 0, 0, -1, -1]], dtype=np.float64)
    hd, sd = torch.from_numpy(h).cuda(), torch.from_numpy(s).cuda()
    I9 = np.eye(9)
    out = host(osk.sketch_cols(dev(I9), 3, 1, 0, h=hd, sigma=sd))
    np.testing.assert_array_equal(unpad(out, 1, 3), ST.T)        # I S_c = S_c
    outT = host(osk.sketch_rows(dev(I9), 3, 1, 0, h=hd, sigma=sd))
    np.testing.assert_array_equal(unpad(outT, 1, 3).T, ST)       # S_c^T I = S_c^T
    outT = host(osk.sketch_rows(dev(I9), 3, 1, 0, h=hd, sigma=sd, workspace=True))
    np.testing.assert_array_equal(unpad(outT, 1, 3).T, ST)


@pytest.mark.parametrize("kept_only", [False, True])
@pytest.mark.parametrize("b", [64, 100, 1024])
def test_sketch_of_identity_is_bit_exact(b, kept_only):
    n, N, e, seed = 700, 3, 2, 17
    keep = synthetic.random_keep(N, e, seed)
    h, s = oracle.hash_tables(seed, N + e, n, b)
    S = oracle.literal_blocks(h, s, b)                       # n x (N+e)*b
    blocks = stored_blocks(N, e, keep, kept_only)
    expect = np.concatenate([S[:, i * b:(i + 1) * b] for i in blocks], axis=1)
    I = dev(np.eye(n))
    out = host(osk.sketch_cols(I, b, N, e, seed=seed, keep=keep, kept_only=kept_only))
    np.testing.assert_array_equal(unpad(out, len(blocks), b), expect)          # I S
    outT = host(osk.sketch_rows(I, b, N, e, seed=seed, keep=keep, kept_only=kept_only))
    np.testing.assert_array_equal(unpad(outT, len(blocks), b).T, expect.T)     # S^T I
    outT = host(osk.sketch_rows(I, b, N, e, seed=seed, keep=keep, kept_only=kept_only,
                                workspace=True))
    np.testing.assert_array_equal(unpad(outT, len(blocks), b).T, expect.T)


@pytest.mark.parametrize("rows,n,b,N,e", [(37, 1003, 100, 3, 2), (256, 4096, 256, 4, 1),
                                          (9, 33, 1, 2, 1), (5, 3000, 1024, 2, 0),
                                          (70, 520, 64, 10, 2)])
def test_sketch_cols_random(rows, n, b, N, e):
    seed = rows + n
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, n)).astype(np.float32)
    out = unpad(host(osk.sketch_cols(dev(X), b, N, e, seed=seed)), N + e, b)
    h, s = oracle.hash_tables(seed, N + e, n, b)
    ref = oracle.sketch_cols(X, h, s, b)
    for i in range(N + e):
        assert rel(out[:, i * b:(i + 1) * b], ref[:, i * b:(i + 1) * b]) <= SKETCH_TOL


@pytest.mark.parametrize("n,cols,b,N,e", [(1003, 77, 100, 3, 2), (4096, 256, 256, 4, 1),
                                          (33, 9, 1, 2, 1), (3000, 40, 1024, 2, 0),
                                          (520, 130, 64, 10, 2)])
def test_sketch_rows_random(n, cols, b, N, e):
    seed = n + cols
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, cols)).astype(np.float32)
    h, s = oracle.hash_tables(seed, N + e, n, b)
    ref = oracle.sketch_rows(X, h, s, b).T                    # cols x (N+e)*b, as unpad gives
    direct = host(osk.sketch_rows(dev(X, ld=cols + 3), b, N, e, seed=seed))
    transposed = host(osk.sketch_rows(dev(X, ld=cols + 3), b, N, e, seed=seed, workspace=True))
    # both paths sum every bucket in ascending k: identical results
    np.testing.assert_array_equal(direct, transposed)
    outT = unpad(transposed, N + e, b)
    for i in range(N + e):
        assert rel(outT[:, i * b:(i + 1) * b], ref[:, i * b:(i + 1) * b]) <= SKETCH_TOL


@pytest.mark.parametrize("n,cols", [(300, 600), (64, 256), (129, 513), (1000, 1024)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_sketch_rows_transposing_tiles(n, cols, dtype):
    # aligned leading dimensions: the transpose takes its whole-tile path
    # (64 x 256 tiles, unguarded vector accesses) inside and its guarded path
    # at the ragged edges; the result must equal the in-place FP32 sketch of
    # the same values bit for bit
    b, N, e = 100, 3, 1
    seed = n + 3 * cols
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, cols)).astype(np.float32)
    Xd = dev(X, ld=(cols + 7) // 8 * 8)
    if dtype == "bf16":
        Xd = Xd.to(torch.bfloat16)
        X = Xd.float().cpu().numpy()          # the BF16 values, exactly
    direct = host(osk.sketch_rows(dev(X, ld=cols + 1), b, N, e, seed=seed))
    transposed = host(osk.sketch_rows(Xd, b, N, e, seed=seed, workspace=True))
    np.testing.assert_array_equal(direct, transposed)
    h, s = oracle.hash_tables(seed, N + e, n, b)
    ref = oracle.sketch_rows(X.astype(np.float64), h, s, b).T
    outT = unpad(transposed, N + e, b)
    assert rel(outT, ref) <= SKETCH_TOL


@pytest.mark.parametrize("n,cols,b,N,e", [
    (20000, 64, 1024, 12, 2),    # 3 windows (the last partial), 2 passes over the blocks
    (9000, 128, 100, 10, 2),     # b < 64-bucket group multiple, 2 windows
    (4100, 36, 256, 4, 0),       # one window, 9 line groups
    (300, 8, 32, 30, 2),         # 32 blocks of one group each
])
def test_sketch_rows_in_place_spread(n, cols, b, N, e):
    # X 16-byte aligned with cols and its leading dimension multiples of 4:
    # the columns are read in place with 16-byte loads and the next window
    # spread over the slots (the whole path's form for such a row-major B);
    # equal bit for bit to the transposing path and within the sketch
    # tolerance of the oracle
    seed = 7 * n + cols
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, cols)).astype(np.float32)
    Xd = dev(X, ld=cols + 4)
    assert Xd.data_ptr() % 16 == 0 and Xd.stride(0) % 4 == 0 and cols % 4 == 0
    direct = host(osk.sketch_rows(Xd, b, N, e, seed=seed))
    transposed = host(osk.sketch_rows(Xd, b, N, e, seed=seed, workspace=True))
    np.testing.assert_array_equal(direct, transposed)
    h, s = oracle.hash_tables(seed, N + e, n, b)
    ref = oracle.sketch_rows(X.astype(np.float64), h, s, b).T
    out = unpad(direct, N + e, b)
    for i in range(N + e):
        assert rel(out[:, i * b:(i + 1) * b], ref[:, i * b:(i + 1) * b]) <= SKETCH_TOL


def _fp32_ascending_sums(X, h, s, b):
    """Every bucket of every block summed in FP32, one rounding per term, in
    ascending k: out[i, c, r] = (...((0 + s[i,k0] X[r,k0]) + s[i,k1] X[r,k1])
    ...) over the k with h[i, k] = c, k0 < k1 < ...  (X: lines x n)."""
    nblk, n = h.shape
    acc = np.zeros((nblk, b, X.shape[0]), np.float32)
    blk = np.arange(nblk)
    for k in range(n):
        acc[blk, h[:, k]] += s[:, k, None].astype(np.float32) * X[None, :, k]
    return acc


@pytest.mark.parametrize("n,b", [
    (20000, 1000),    # block stride <= 1024: lists built by 16 waves per region
    (20000, 1500),    # <= 2048: 8 waves per region
    (9500, 2500),     # > 2048: one wave per region
])
def test_sketch_sums_each_bucket_in_ascending_k(n, b):
    # The bucket lists hold every bucket's positions in ascending k (any
    # number of waves builds the same lists), and the sketch kernel adds a
    # bucket's terms in list order across the windows: the FP32 sketch
    # equals the FP32 sum taken term by term in ascending k, bit for bit,
    # reading rows (A S) and reading columns in place (S^T B).
    N, e, seed = 2, 1, n + b
    rng = np.random.default_rng(seed)
    h, s = oracle.hash_tables(seed, N + e, n, b)
    X = rng.standard_normal((8, n)).astype(np.float32)
    ref = _fp32_ascending_sums(X, h, s, b)
    out = unpad(host(osk.sketch_cols(dev(X), b, N, e, seed=seed)), N + e, b)
    for i in range(N + e):
        np.testing.assert_array_equal(out[:, i * b:(i + 1) * b], ref[i].T)
    Y = rng.standard_normal((n, 12)).astype(np.float32)
    Yd = dev(Y, ld=16)
    assert Yd.data_ptr() % 16 == 0
    ref = _fp32_ascending_sums(np.ascontiguousarray(Y.T), h, s, b)
    out = unpad(host(osk.sketch_rows(Yd, b, N, e, seed=seed)), N + e, b)
    for i in range(N + e):
        np.testing.assert_array_equal(out[:, i * b:(i + 1) * b], ref[i].T)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp8", "fp8x3"])
def test_whole_path_row_major_b_in_place_equals_column_major(precision):
    # a row-major B whose columns are sketched in place and the same values
    # given column-major (B^T's rows, read directly): the same sketch sums,
    # so the same C bit for bit, in every operand precision
    m, n, l, b, N, e = 96, 9000, 136, 256, 4, 1
    rng = np.random.default_rng(31)
    A = rng.standard_normal((m, n)).astype(np.float32)
    B = rng.standard_normal((n, l)).astype(np.float32)
    keep = synthetic.random_keep(N, e, 31)
    Bd = dev(B)
    Bcm = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t()     # column-major view
    assert Bd.stride(1) == 1 and Bcm.stride(0) == 1
    C1 = host(osk.matmul(dev(A), Bd, b, N, e, seed=5, keep=keep, precision=precision))
    C2 = host(osk.matmul(dev(A), Bcm, b, N, e, seed=5, keep=keep, precision=precision))
    np.testing.assert_array_equal(C1, C2)


def test_sketch_cols_is_deterministic():
    X = dev(np.random.default_rng(3).standard_normal((64, 5000)))
    a = host(osk.sketch_cols(X, 256, 4, 1, seed=3))
    b = host(osk.sketch_cols(X, 256, 4, 1, seed=3))
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------------------
# grouped product over kept blocks
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,l,b,nst", [(256, 256, 256, 5), (300, 77, 100, 3), (1, 1, 32, 1),
                                       (513, 255, 64, 4), (64, 700, 1024, 2)])
def test_gemm_kept_vs_oracle(m, l, b, nst):
    rng = np.random.default_rng(m * 7 + l)
    bp = osk.block_stride(b)
    At = np.zeros((m, nst * bp), np.float32)        # line-major sketch of A
    Bt = np.zeros((l, nst * bp), np.float32)        # line-major sketch of B
    for j in range(nst):
        At[:, j * bp:j * bp + b] = rng.standard_normal((m, b))
        Bt[:, j * bp:j * bp + b] = rng.standard_normal((l, b))
    keep = np.ones(nst, np.uint8)
    if nst > 1:
        keep[rng.integers(nst)] = 0
    C = host(osk.gemm_kept(dev(At), dev(Bt), b, keep=keep))
    ref = oracle.block_product(unpad(At, nst, b), unpad(Bt, nst, b).T, b, keep)
    assert rel(C, ref) <= PRODUCT_TOL


# ---------------------------------------------------------------------------
# the whole path
# ---------------------------------------------------------------------------

def _matmul_case(m, n, l, b, N, e, seed, keep, kept_only, col_major, data="gauss"):
    if data == "gauss":
        A, B = synthetic.gaussian_pair(m, n, l, seed)
    else:
        A, B = synthetic.lowrank_pair(m, n, l, seed, rank=8)
    Ad = dev(A)
    if col_major:
        Bd = dev(B.T).t()              # n x l view with unit row stride
    else:
        Bd = dev(B, ld=l + 1)
    C = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep, kept_only=kept_only))
    ref = oracle.sketched_matmul(A, B, b, N, e, seed=seed, keep=keep)
    return C, ref, A, B


@pytest.mark.parametrize("kept_only", [False, True])
@pytest.mark.parametrize("col_major", [False, True])
def test_matmul_config1(kept_only, col_major):
    # 256x4096 by 4096x256, b=256, N=4, e=1, one random block dropped.
    seed = 1
    keep = synthetic.random_keep(4, 1, seed)
    C, ref, _, _ = _matmul_case(256, 4096, 256, 256, 4, 1, seed, keep, kept_only, col_major)
    assert rel(C, ref) <= PRODUCT_TOL


@pytest.mark.parametrize("m,n,l,b,N,e,drop", [
    (300, 1001, 77, 100, 3, 1, 1),     # ragged everywhere
    (513, 2050, 257, 64, 4, 2, 3),     # more losses than provisioned (K < N)
    (129, 777, 384, 32, 2, 2, 0),      # K > N: all N+e kept
    (1, 50, 1, 1, 1, 0, 0),            # degenerate sizes
    (40, 3, 33, 8, 2, 1, 1),           # n < b
    (70, 20000, 33, 8192, 2, 1, 1),    # the largest b: two sketch passes
    (50, 5000, 40, 128, 190, 10, 7),   # 200 blocks: three sketch passes
])
def test_matmul_ragged_and_masks(m, n, l, b, N, e, drop):
    seed = m + n
    keep = synthetic.random_keep(N, e, seed, drop=drop)
    for kept_only in (False, True):
        C, ref, _, _ = _matmul_case(m, n, l, b, N, e, seed, keep, kept_only, col_major=False)
        assert rel(C, ref) <= PRODUCT_TOL, (kept_only, rel(C, ref))


@pytest.mark.parametrize("m,n,l,b,N,e,drop", [
    (256, 4096, 256, 256, 4, 1, 1),    # one tile, 32 K steps: 16 splits of one step pair
    (300, 2000, 77, 100, 3, 2, 1),     # two tiles, bp = 128: 4 steps per block
    (100, 3000, 520, 96, 5, 0, 0),     # 15 steps: splits of 4, the last one odd (3)
    (1, 64, 1, 32, 1, 0, 0),           # one step: no split
])
def test_matmul_split_k(m, n, l, b, N, e, drop):
    # products with few tiles split their K loop over several workgroups
    # per tile (partials summed in split order): against the oracle, against
    # the unsplit block product of the same sketches, and run to run
    seed = 5 * m + l
    keep = synthetic.random_keep(N, e, seed, drop=drop)
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    Ad, Bd = dev(A), dev(B)
    C1 = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep))
    C2 = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep))
    np.testing.assert_array_equal(C1, C2)
    ref = oracle.sketched_matmul(A, B, b, N, e, seed=seed, keep=keep)
    assert rel(C1, ref) <= PRODUCT_TOL
    At = osk.sketch_cols(Ad, b, N, e, seed=seed)
    Bt = osk.sketch_rows(Bd, b, N, e, seed=seed)
    unsplit = host(osk.gemm_kept(At, Bt, b, keep=keep))      # os_gemm_kept never splits
    assert rel(C1, unsplit) <= 1e-6


def test_matmul_exact_with_permutation_sketch():
    # b = n and h a permutation in every block: S_i S_i^T = I, C = AB.
    m, n, l, N = 96, 256, 80, 2
    rng = np.random.default_rng(4)
    A, B = synthetic.gaussian_pair(m, n, l, 4)
    h = np.stack([rng.permutation(n) for _ in range(N)]).astype(np.int32)
    s = rng.choice(np.array([-1, 1], np.int8), size=(N, n))
    C = host(osk.matmul(dev(A), dev(B), n, N, 0, h=torch.from_numpy(h).cuda(),
                        sigma=torch.from_numpy(s).cuda()))
    AB = A.astype(np.float64) @ B.astype(np.float64)
    assert rel(C, AB) <= PRODUCT_TOL


def test_kept_only_equals_faithful():
    m, n, l, b, N, e, seed = 200, 3000, 150, 128, 4, 2, 8
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    keep = synthetic.random_keep(N, e, seed)
    c1 = host(osk.matmul(dev(A), dev(B), b, N, e, seed=seed, keep=keep, kept_only=False))
    c2 = host(osk.matmul(dev(A), dev(B), b, N, e, seed=seed, keep=keep, kept_only=True))
    assert rel(c1, c2) <= 1e-6


def test_error_paths_raise():
    A = dev(np.ones((4, 16)))
    B = dev(np.ones((16, 4)))
    with pytest.raises(osk.OversketchError):
        osk.matmul(A, B, 4, 2, 1, keep=np.zeros(3, np.uint8))
    with pytest.raises(osk.OversketchError):
        osk.matmul(A, B, 0, 2, 1)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(osk.OversketchError):
        osk.matmul(A, B, 4, 2, 1, workspace=small)


# ---------------------------------------------------------------------------
# per-C-block keep masks (each b x b block of C keeps its own workers)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,l,b,N,e", [(600, 2048, 520, 256, 3, 2),   # tiles = blocks
                                         (300, 1001, 250, 100, 3, 1),   # block < tile
                                         (700, 1500, 640, 300, 2, 2),   # 2 tiles per block side
                                         (200, 700, 230, 96, 3, 1)])    # odd steps per block
def test_matmul_per_block_masks(m, n, l, b, N, e):
    seed = m + l
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    rng = np.random.default_rng(seed)
    nbI, nbJ = -(-m // b), -(-l // b)
    cmask = (rng.random((nbI, nbJ, N + e)) < 0.6).astype(np.uint8)
    cmask[0, 0, :] = 0                      # a block every worker missed: zero
    cmask[-1, -1, :] = 1                    # a block that kept all N+e (K > N)
    if nbJ > 1:
        cmask[0, 1, :] = 0
        cmask[0, 1, 0] = 1                  # a block with one worker (K < N)
    C = host(osk.matmul_cmask(dev(A), dev(B, ld=l + 1), b, N, e, cmask, seed=seed))
    ref = oracle.sketched_matmul_cmask(A, B, b, N, e, cmask, seed=seed)
    assert np.all(C[:b, :b] == 0)
    assert rel(C, ref) <= PRODUCT_TOL
    # a uniform mask reproduces the global-mask block product exactly (the
    # unsplit os_gemm_kept on the same sketches), and the whole path, whose
    # K loop is split for these few tiles (another summation order), to
    # rounding
    keep = synthetic.random_keep(N, e, seed)
    uni = np.broadcast_to(keep, (nbI, nbJ, N + e)).copy()
    Ad, Bd = dev(A), dev(B, ld=l + 1)
    Cu = host(osk.matmul_cmask(Ad, Bd, b, N, e, uni, seed=seed))
    Cg = host(osk.gemm_kept(osk.sketch_cols(Ad, b, N, e, seed=seed),
                            osk.sketch_rows(Bd, b, N, e, seed=seed), b, keep=keep))
    np.testing.assert_array_equal(Cu, Cg)
    Cw = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep))
    assert rel(Cw, Cg) <= 1e-6


# ---------------------------------------------------------------------------
# os_matmul_ex: column-major A, BF16 operands in either layout
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,l,b,N,e", [(300, 1001, 77, 100, 3, 1), (96, 4096, 130, 256, 4, 0)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("kept_only", [False, True])
def test_matmul_ex_column_major_a(m, n, l, b, N, e, dtype, kept_only):
    seed = m + l
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    keep = synthetic.random_keep(N, e, seed)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    # A stored as X = A^T (n x m, row-major), passed as the column-major view
    X = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().to(tdt)
    Bd = torch.from_numpy(B).cuda().to(tdt)
    C = host(osk.matmul_ex(X.t(), Bd, b, N, e, seed=seed, keep=keep, kept_only=kept_only))
    Av = X.t().float().cpu().numpy()        # the values the library read
    Bv = Bd.float().cpu().numpy()
    ref = oracle.sketched_matmul(Av, Bv, b, N, e, seed=seed, keep=keep)
    assert rel(C, ref) <= PRODUCT_TOL


def test_matmul_ex_matches_matmul():
    m, n, l, b, N, e, seed = 200, 2048, 150, 128, 4, 1, 9
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C1 = host(osk.matmul(Ad, Bd, b, N, e, seed=seed))
    C2 = host(osk.matmul_ex(Ad, Bd, b, N, e, seed=seed))
    np.testing.assert_array_equal(C1, C2)


def _in_layout(X, col_major, dtype):
    """X (rows x cols, host) as a CUDA tensor of dtype, row-major or as the
    transposed view of a row-major X^T (column-major)."""
    t = torch.from_numpy(np.ascontiguousarray(X.T if col_major else X)).cuda().to(dtype)
    return t.t() if col_major else t


@pytest.mark.parametrize("n", [2048, 1001])
@pytest.mark.parametrize("a_cm,b_cm", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("types", [("bf16", "bf16"), ("bf16", "f32"), ("f32", "bf16")])
def test_matmul_ex_bf16_any_layout(n, a_cm, b_cm, types):
    # a BF16 operand in either layout (sketched in place, or transposed as
    # BF16 first) gives the FP32 path's result on its converted values, bit
    # for bit; n = 1001 takes the unaligned loads
    m, l, b, N, e, seed = 200, 150, 128, 4, 1, n + 2 * a_cm + b_cm
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    dt = {"bf16": torch.bfloat16, "f32": torch.float32}
    Ax = _in_layout(A, a_cm, dt[types[0]])
    Bx = _in_layout(B, b_cm, dt[types[1]])
    C = host(osk.matmul_ex(Ax, Bx, b, N, e, seed=seed))
    ref = host(osk.matmul_ex(_in_layout(Ax.float().cpu().numpy(), a_cm, torch.float32),
                             _in_layout(Bx.float().cpu().numpy(), b_cm, torch.float32),
                             b, N, e, seed=seed))
    np.testing.assert_array_equal(C, ref)
    if types == ("bf16", "bf16") and n == 1001:
        o = oracle.sketched_matmul(Ax.float().cpu().numpy(), Bx.float().cpu().numpy(), b, N, e,
                                   seed=seed)
        assert rel(C, o) <= PRODUCT_TOL

# ---------------------------------------------------------------------------
# grouped bucket order (the whole path's prepared sketch)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,b,N,e", [(32768, 1024, 8, 2), (9001, 100, 3, 1), (20000, 2048, 2, 1),
                                     (3000, 64, 2, 2), (5000, 1, 2, 0), (70000, 300, 2, 1)])
def test_grouped_order_is_a_permutation_per_block(n, b, N, e):
    seed = n + b
    bp = osk.block_stride(b)
    nat = osk.sketch_prepare(n, b, N, e, seed=seed)
    np.testing.assert_array_equal(osk.bucket_order(nat, n, b, N, e, seed=seed).cpu().numpy(),
                                  np.tile(np.arange(bp), (N + e, 1)))
    grp = osk.sketch_prepare(n, b, N, e, seed=seed, grouped=True)
    order = osk.bucket_order(grp, n, b, N, e, seed=seed).cpu().numpy()
    for i in range(N + e):
        np.testing.assert_array_equal(np.sort(order[i, :b]), np.arange(b))
        np.testing.assert_array_equal(order[i, b:], np.arange(b, bp))
    # the order is a function of the sketch (reproducible)
    grp2 = osk.sketch_prepare(n, b, N, e, seed=seed, grouped=True)
    np.testing.assert_array_equal(osk.bucket_order(grp2, n, b, N, e, seed=seed).cpu().numpy(),
                                  order)


@pytest.mark.parametrize("n,b,N,e,kept_only", [(20000, 256, 4, 2, False), (9001, 100, 3, 1, True),
                                               (40000, 1024, 3, 1, False)])
def test_grouped_sketches_are_the_natural_ones_permuted(n, b, N, e, kept_only):
    # the same sums (each bucket in ascending k), at the columns the order
    # names: bit-exact, both sketch kinds
    seed = 3 * n + b
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((37, n)).astype(np.float32)
    Y = rng.standard_normal((n, 29)).astype(np.float32)
    keep = synthetic.random_keep(N, e, seed)
    bp = osk.block_stride(b)
    nat = osk.sketch_prepare(n, b, N, e, seed=seed)
    grp = osk.sketch_prepare(n, b, N, e, seed=seed, grouped=True)
    order = osk.bucket_order(grp, n, b, N, e, seed=seed).cpu().numpy()
    stored = stored_blocks(N, e, keep, kept_only)
    for fn, M, kw in ((osk.sketch_cols, X, {}), (osk.sketch_rows, Y, {"workspace": True})):
        a = host(fn(dev(M), b, N, e, seed=seed, keep=keep, kept_only=kept_only, prep=nat, **kw))
        g = host(fn(dev(M), b, N, e, seed=seed, keep=keep, kept_only=kept_only, prep=grp, **kw))
        for j, i in enumerate(stored):
            np.testing.assert_array_equal(g[:, j * bp:(j + 1) * bp],
                                          a[:, j * bp + order[i]])


@pytest.mark.parametrize("n,b,N,e", [(32768, 1024, 8, 2), (65536, 512, 4, 1), (20000, 2048, 3, 0)])
def test_grouped_order_walks_less_padding(n, b, N, e):
    seed = 2 + n
    nat = osk.sketch_prepare(n, b, N, e, seed=seed)
    grp = osk.sketch_prepare(n, b, N, e, seed=seed, grouped=True)
    w_nat, real = osk.list_entries(nat, n, b, N, e, seed=seed)
    w_grp, real2 = osk.list_entries(grp, n, b, N, e, seed=seed)
    assert real == real2 == (N + e) * n
    assert real <= w_grp < w_nat, (w_nat / real, w_grp / real)


def _grouped_order_reference(h, n, b, win=8192):
    """The library's grouping written plainly: D levels of a k-d split of the
    ceil(b/64) groups; level d sorts each node's buckets by their count in the
    windows w = d (mod D), ties by current position (a stable sort)."""
    G = (b + 63) // 64
    D = 0
    while (1 << D) < G:
        D += 1
    nwin = (n + win - 1) // win
    at = np.arange(b)
    for d in range(D):
        feat = np.zeros(b, np.int64)
        for w in range(d, nwin, D):
            feat += np.bincount(h[w * win:min(n, (w + 1) * win)], minlength=b)
        node = np.zeros(b, np.int64)
        for p in range(b):
            glo, ghi = 0, G
            for _ in range(d):
                gm = (glo + ghi) >> 1
                if (p >> 6) < gm:
                    ghi = gm
                else:
                    glo = gm
            node[p] = glo
        order = np.lexsort((np.arange(b), feat[at], node))
        at = at[order]
    return at


@pytest.mark.parametrize("n,b,N,e", [(32768, 1024, 3, 1), (9001, 100, 2, 1), (20000, 2048, 2, 0),
                                     (70000, 300, 2, 1), (16384, 4100, 1, 1)])
def test_grouped_order_follows_its_definition(n, b, N, e):
    seed = 7 * n + b
    grp = osk.sketch_prepare(n, b, N, e, seed=seed, grouped=True)
    order = osk.bucket_order(grp, n, b, N, e, seed=seed).cpu().numpy()
    h, _ = oracle.hash_tables(seed, N + e, n, b)
    for i in range(N + e):
        np.testing.assert_array_equal(order[i, :b], _grouped_order_reference(h[i], n, b))
