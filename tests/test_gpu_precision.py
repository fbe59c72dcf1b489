"""GPU parity of the reduced-precision block product (BF16 operands, FP32
accumulation; the split form adds the residual terms), through the C ABI.

  - quantization: bit-exact against the oracle's round-to-nearest-even
    definition applied to the same FP32 sketch values;
  - block product on BF16 inputs: the products of BF16 values are exact, so
    only FP32 accumulation separates it from the FP64 sum: <= 1e-5 relative
    Frobenius, as for the FP32 path;
  - whole path against the FP64 oracle on the same sketch: within the error
    the arithmetic allows.  Each operand is rounded once, relatively by at
    most u = 2^-8 (BF16: 8 significant bits), so
    |C - C_o| <= (2u + u^2) (|A~| |B~|^T) / K entrywise, plus FP32 terms;
    the split form leaves u_s = 2^-16 per operand instead.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1811_02653_amd as osk  # noqa: E402

U_BF16 = 2.0 ** -8
U_SPLIT = 2.0 ** -16
FP32_TOL = 1e-5
FP8_BLOCK = 64          # values per E8M0 scale


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def line_major_sketch(rng, lines, b, nst):
    """A line-major FP32 sketch with zero padding columns."""
    bp = osk.block_stride(b)
    S = np.zeros((lines, nst * bp), np.float32)
    for j in range(nst):
        S[:, j * bp:j * bp + b] = rng.standard_normal((lines, b)) * np.exp(rng.standard_normal())
    return S


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("lines,b,nst", [(37, 100, 3), (256, 256, 5), (5, 1, 2), (64, 1024, 2)])
def test_quantize_bf16_bit_exact(lines, b, nst, split):
    rng = np.random.default_rng(lines + b)
    S = line_major_sketch(rng, lines, b, nst)
    prec = "bf16x3" if split else "bf16"
    Q = host(osk.sketch_quantize(torch.from_numpy(S).cuda(), b, nst, precision=prec))
    bp, bq = osk.block_stride(b), osk.block_stride_prec(b, prec)
    assert bq % 64 == 0 and bq >= b
    zq = nst * bq
    assert Q.shape == (lines, zq * (2 if split else 1))
    for j in range(nst):
        x = S[:, j * bp:j * bp + b]
        hi, lo = oracle.bf16_split(x)
        np.testing.assert_array_equal(Q[:, j * bq:j * bq + b], hi)
        assert np.all(Q[:, j * bq + b:(j + 1) * bq] == 0)
        if split:
            np.testing.assert_array_equal(Q[:, zq + j * bq:zq + j * bq + b], lo)
            assert np.all(Q[:, zq + j * bq + b:zq + (j + 1) * bq] == 0)


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("m,l,b,nst", [(256, 256, 256, 5), (300, 77, 100, 3), (1, 1, 32, 1),
                                       (513, 255, 64, 4), (64, 700, 1024, 2)])
def test_gemm_kept_bf16_vs_fp64(m, l, b, nst, split):
    rng = np.random.default_rng(m * 7 + l)
    prec = "bf16x3" if split else "bf16"
    SA = line_major_sketch(rng, m, b, nst)
    SB = line_major_sketch(rng, l, b, nst)
    keep = np.ones(nst, np.uint8)
    if nst > 1:
        keep[rng.integers(nst)] = 0
    QA = osk.sketch_quantize(torch.from_numpy(SA).cuda(), b, nst, precision=prec)
    QB = osk.sketch_quantize(torch.from_numpy(SB).cuda(), b, nst, precision=prec)
    C = host(osk.gemm_kept_prec(QA, QB, b, nst, precision=prec, keep=keep))
    # reference: FP64 sums of the exact products of the BF16 values
    qa, qb = host(QA), host(QB)
    bq = osk.block_stride_prec(b, prec)
    zq = nst * bq
    ref = np.zeros((m, l))
    for j in np.flatnonzero(keep):
        a, bb = qa[:, j * bq:(j + 1) * bq], qb[:, j * bq:(j + 1) * bq]
        ref += a @ bb.T
        if split:
            ref += a @ qb[:, zq + j * bq:zq + (j + 1) * bq].T
            ref += qa[:, zq + j * bq:zq + (j + 1) * bq] @ bb.T
    ref /= keep.sum()
    assert oracle.rel_frob(C, ref) <= FP32_TOL


def _bound(A, B, b, N, e, seed, keep):
    """|| |A~| |B~|^T / K ||_F on the oracle's own sketch."""
    h, s = oracle.hash_tables(seed, N + e, A.shape[1], b)
    At = np.abs(oracle.sketch_cols(A, h, s, b))
    Bt = np.abs(oracle.sketch_rows(B, h, s, b))
    return np.sqrt(oracle.frob2(oracle.block_product(At, Bt, b, keep)))


@pytest.mark.parametrize("m,n,l,b,N,e", [(256, 4096, 256, 256, 4, 1), (300, 1001, 77, 100, 3, 1),
                                         (40, 3, 33, 8, 2, 1)])
def test_matmul_bf16_within_rounding_bound(m, n, l, b, N, e):
    seed = m + n
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    keep = synthetic.random_keep(N, e, seed)
    ref = oracle.sketched_matmul(A, B, b, N, e, seed=seed, keep=keep)
    bound = _bound(A, B, b, N, e, seed, keep)
    nref = np.sqrt(oracle.frob2(ref))
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    errs = {}
    for prec, u in (("bf16", U_BF16), ("bf16x3", U_SPLIT)):
        C = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep, precision=prec))
        err = np.sqrt(oracle.frob2(C - ref))
        errs[prec] = err
        assert err <= (2 * u + u * u) * bound + FP32_TOL * nref, (prec, err, bound)
    # the residual terms do recover accuracy
    assert errs["bf16x3"] < errs["bf16"] / 16


@pytest.mark.parametrize("precision", ["bf16", "bf16x3", "fp8", "fp8x3"])
@pytest.mark.parametrize("m,n,l,b,N,e,kept_only", [(300, 1001, 77, 100, 3, 1, False),
                                                   (256, 4096, 256, 256, 4, 1, True),
                                                   (130, 2500, 90, 64, 2, 2, False),
                                                   (70, 9000, 40, 1000, 2, 1, True),
                                                   # 320 groups of 64 buckets: two sketch
                                                   # passes of 20 slots per wave
                                                   (40, 3000, 37, 2048, 8, 2, False),
                                                   # 12 x 11 = 132 tiles: no split K loop
                                                   (3072, 1500, 2816, 128, 2, 1, False)])
def test_matmul_fused_quantization_is_the_staged_path(m, n, l, b, N, e, kept_only, precision):
    # the whole path rounds each sketch to BF16 (or quantizes it to FP8 with
    # its block scales, when b rounded up to 64 is a multiple of 128; b = 64
    # takes the staged path) in the sketch's epilogue; it must give what the
    # staged path gives (FP32 sketches, then their low-precision copies, then
    # the block product): bit for bit when the product has enough tiles to
    # run unsplit, and to FP32 rounding of the same terms summed in another
    # order (1e-5, the product tolerance; up to 61440 terms here) when the
    # whole path splits its K loop over several workgroups per tile
    seed = m + n + b
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    keep = synthetic.random_keep(N, e, seed)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep, kept_only=kept_only,
                        precision=precision))
    nst = osk.stored_count(N, e, keep, kept_only)
    prep = osk.sketch_prepare(n, b, N, e, seed=seed)
    At = osk.sketch_cols(Ad, b, N, e, seed=seed, keep=keep, kept_only=kept_only, prep=prep)
    Bt = osk.sketch_rows(Bd, b, N, e, seed=seed, keep=keep, kept_only=kept_only, prep=prep,
                         workspace=True)
    QA = osk.sketch_quantize(At, b, nst, precision=precision)
    QB = osk.sketch_quantize(Bt, b, nst, precision=precision)
    C2 = host(osk.gemm_kept_prec(QA, QB, b, nst, precision=precision,
                                 keep=None if kept_only else keep))
    if -(-m // 256) * -(-l // 256) > 128:
        np.testing.assert_array_equal(C, C2)
    else:
        assert oracle.rel_frob(C, C2) <= 1e-5


# ---------------------------------------------------------------------------
# FP8 E4M3 with one E8M0 scale per 64 values
# ---------------------------------------------------------------------------

def decode_fp8(Q, b, nst, split):
    """(values, exponents) of a quantized FP8 copy: the E4M3 codes of each
    row times 2^s of their 64-value block (FP64), and the block exponents."""
    Q = np.asarray(Q, dtype=np.uint8)
    bq = osk.block_stride_prec(b, "fp8")
    ncode = nst * bq * (2 if split else 1)
    codes = Q[:, :ncode].astype(np.int64)
    s = Q[:, ncode:ncode + ncode // FP8_BLOCK].astype(np.int64) - 127
    mag = oracle.e4m3_values()[codes & 0x7F]
    val = np.where(codes & 0x80, -mag, mag) * np.repeat(np.ldexp(1.0, s), FP8_BLOCK, axis=1)
    return val, s


def host_u8(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("lines,b,nst", [(37, 100, 3), (256, 256, 5), (5, 1, 2), (64, 1024, 2)])
def test_quantize_fp8_bit_exact(lines, b, nst, split):
    rng = np.random.default_rng(lines + b + 1)
    S = line_major_sketch(rng, lines, b, nst)
    prec = "fp8x3" if split else "fp8"
    Q = host_u8(osk.sketch_quantize(torch.from_numpy(S).cuda(), b, nst, precision=prec))
    assert Q.shape == (lines, osk.quantized_row(b, nst, prec))
    bp, bq = osk.block_stride(b), osk.block_stride_prec(b, prec)
    assert bq % 128 == 0 and bq >= b
    # the oracle's quantization of the same FP32 values, in the copy's layout
    X = np.zeros((lines, nst * bq))
    for j in range(nst):
        X[:, j * bq:j * bq + b] = S[:, j * bp:j * bp + b]
    hi, s_hi = oracle.fp8_block_quantize(X, FP8_BLOCK)
    val, s = decode_fp8(Q, b, nst, split)
    zq = nst * bq
    np.testing.assert_array_equal(val[:, :zq], hi)
    np.testing.assert_array_equal(s[:, :zq // FP8_BLOCK], s_hi)
    if split:
        lo, s_lo = oracle.fp8_block_quantize(X - hi, FP8_BLOCK)
        np.testing.assert_array_equal(val[:, zq:], lo)
        np.testing.assert_array_equal(s[:, zq // FP8_BLOCK:], s_lo)


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("m,l,b,nst", [(256, 256, 256, 5), (300, 77, 100, 3), (1, 1, 32, 1),
                                       (513, 255, 64, 4), (64, 700, 1024, 2), (300, 520, 1024, 4),
                                       (257, 129, 2048, 3)])
def test_gemm_kept_fp8_vs_fp64(m, l, b, nst, split):
    rng = np.random.default_rng(m * 5 + l)
    prec = "fp8x3" if split else "fp8"
    SA = line_major_sketch(rng, m, b, nst)
    SB = line_major_sketch(rng, l, b, nst)
    keep = np.ones(nst, np.uint8)
    if nst > 1:
        keep[rng.integers(nst)] = 0
    QA = osk.sketch_quantize(torch.from_numpy(SA).cuda(), b, nst, precision=prec)
    QB = osk.sketch_quantize(torch.from_numpy(SB).cuda(), b, nst, precision=prec)
    C = host(osk.gemm_kept_prec(QA, QB, b, nst, precision=prec, keep=keep))
    # reference: FP64 sums of the exact products of the scaled FP8 values
    qa, _ = decode_fp8(host_u8(QA), b, nst, split)
    qb, _ = decode_fp8(host_u8(QB), b, nst, split)
    bq = osk.block_stride_prec(b, prec)
    zq = nst * bq
    ref = np.zeros((m, l))
    mag = np.zeros((m, l))
    for j in np.flatnonzero(keep):
        a, bb = qa[:, j * bq:(j + 1) * bq], qb[:, j * bq:(j + 1) * bq]
        ref += a @ bb.T
        mag += np.abs(a) @ np.abs(bb).T
        if split:
            alo, blo = qa[:, zq + j * bq:zq + (j + 1) * bq], qb[:, zq + j * bq:zq + (j + 1) * bq]
            ref += a @ blo.T + alo @ bb.T
            mag += np.abs(a) @ np.abs(blo).T + np.abs(alo) @ np.abs(bb).T
    K = keep.sum()
    ref /= K
    mag /= K
    # The scaled FP8 MFMA sums 64 exact products per instruction before adding
    # them to the FP32 accumulator.  That inner sum is not exact FP32: on
    # gfx950 it carries about 16 significant bits (1.5e-5 relative measured
    # against the exact FP64 sum of the same FP8 products).  Allow 2^-14 of
    # the products' magnitude for it, plus one FP32 ulp per accumulation.
    steps = K * (bq // 64) * (3 if split else 1)
    err = np.sqrt(oracle.frob2(C - ref))
    bound = (2.0 ** -14 + steps * 2.0 ** -23) * np.sqrt(oracle.frob2(mag))
    assert err <= bound, (err, bound, oracle.rel_frob(C, ref))
    # and it stays far below the FP8 rounding of the operands (2^-4)
    assert oracle.rel_frob(C, ref) <= 1e-4


def _bound_fp8(A, B, b, N, e, seed, keep, u):
    """|| Ahat Bhat^T / K ||_F with Ahat = |A~| + 2^-10/224 * blockmax / u:
    the FP8 rounding of an element is at most u |x| + blockmax / 229376
    (blocks of 64 values along each row of the line-major sketch, as the
    quantized copy lays them out: the bound only needs blockmax >= the
    block's true maximum, which a 64-block of the unpadded layout is not;
    blocks of 32 of the unpadded row give a smaller maximum, so the row
    maximum is used)."""
    h, s = oracle.hash_tables(seed, N + e, A.shape[1], b)
    At = oracle.sketch_cols(A, h, s, b)
    Bt = oracle.sketch_rows(B, h, s, b).T

    def hat(X):
        Xa = np.abs(X)
        rowmax = Xa.max(axis=1, keepdims=True)
        return Xa + rowmax / 229376.0 / u

    return np.sqrt(oracle.frob2(oracle.block_product(hat(At), hat(Bt).T, b, keep)))


@pytest.mark.parametrize("m,n,l,b,N,e", [(256, 4096, 256, 256, 4, 1), (300, 1001, 77, 100, 3, 1),
                                         (300, 2600, 77, 1024, 3, 1)])
def test_matmul_fp8_within_rounding_bound(m, n, l, b, N, e):
    seed = m + n
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    keep = synthetic.random_keep(N, e, seed)
    ref = oracle.sketched_matmul(A, B, b, N, e, seed=seed, keep=keep)
    nref = np.sqrt(oracle.frob2(ref))
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    u = 2.0 ** -4
    C = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep, precision="fp8"))
    err = np.sqrt(oracle.frob2(C - ref))
    assert err <= (2 * u + u * u) * _bound_fp8(A, B, b, N, e, seed, keep, u) + FP32_TOL * nref
    C3 = host(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep, precision="fp8x3"))
    err3 = np.sqrt(oracle.frob2(C3 - ref))
    # the residual pass recovers about four more bits
    assert err3 < err / 8


# ---------------------------------------------------------------------------
# The precision workload: the small validation shapes (A 256 x 4096,
# B 4096 x 256, b = 256, N = 4, e = 1, one block dropped) with log-normal
# (sigma = 2) row norms of A and column norms of B.  Line norms spread over
# about five decades, so one scale per tensor would leave the small lines
# with few significant bits; the per-64-value power-of-two scales of the
# FP8 copies (and BF16's own exponent) keep every line's relative accuracy.
# Each entry of C is checked against the oracle's FP64 sketched product on
# the same S, within the rounding bound of its own operands:
#   |C - C_o|[r,c] <= ((1+u)^2 - 1 + g) * M[r,c] + (FP8) subnormal terms,
#   M = (|A~| |B~|^T) / K on the oracle's sketch, g = FP32 accumulation
#   (K * stride * 2^-24, a worst case) plus, for FP8, the scaled MFMA's
#   inner sum (2^-14 of the products' magnitude, see test_gemm_kept_fp8_vs_fp64).
# ---------------------------------------------------------------------------

LOGNORMAL_CASE = dict(m=256, n=4096, l=256, b=256, N=4, e=1)


@pytest.fixture(scope="module")
def lognormal_case():
    c = LOGNORMAL_CASE
    seed = 3
    A, B = synthetic.lognormal_scaled_pair(c["m"], c["n"], c["l"], seed, sigma=2.0)
    keep = synthetic.random_keep(c["N"], c["e"], seed)
    assert keep.sum() == c["N"]
    h, s = oracle.hash_tables(seed, c["N"] + c["e"], c["n"], c["b"])
    At = oracle.sketch_cols(A, h, s, c["b"])
    Bt = oracle.sketch_rows(B, h, s, c["b"])
    ref = oracle.block_product(At, Bt, c["b"], keep)
    # the same as the oracle's whole path
    np.testing.assert_array_equal(
        ref, oracle.sketched_matmul(A, B, c["b"], c["N"], c["e"], seed=seed, keep=keep))
    return dict(A=A, B=B, seed=seed, keep=keep, At=At, Bt=Bt, ref=ref)


def test_lognormal_inputs_span_decades(lognormal_case):
    # the workload is what it claims: line norms spread over >= 4 decades
    ra = np.linalg.norm(lognormal_case["A"], axis=1)
    cb = np.linalg.norm(lognormal_case["B"], axis=0)
    assert ra.max() / ra.min() > 1e4 and cb.max() / cb.min() > 1e4


@pytest.mark.parametrize("precision,u", [("fp32", 0.0), ("bf16", 2.0 ** -8),
                                         ("bf16x3", 2.0 ** -16), ("fp8", 2.0 ** -4),
                                         ("fp8x3", 2.0 ** -8)])
def test_lognormal_norms_entrywise_rounding_bound(lognormal_case, precision, u):
    c, d = LOGNORMAL_CASE, lognormal_case
    b, K = c["b"], int(d["keep"].sum())
    Ad, Bd = torch.from_numpy(d["A"]).cuda(), torch.from_numpy(d["B"]).cuda()
    C = host(osk.matmul(Ad, Bd, b, c["N"], c["e"], seed=d["seed"], keep=d["keep"],
                        precision=precision))
    ref = d["ref"]
    Aa, Ba = np.abs(d["At"]), np.abs(d["Bt"])
    fp8 = precision.startswith("fp8")
    if fp8:
        # an element's FP8 rounding is at most u |x| + c, c = (its 64-block
        # max) / 229376 (the subnormal step; the line's maximum stands in for
        # the block's).  Split form: |x - hi - lo| <= u_h (u_h |x| + c) + c_lo
        # with c_lo <= u_h * blockmax / 229376, so u = u_h^2 = 2^-8 and an
        # absolute term 2 u_h c.  Writing the absolute term as u * (c' / u)
        # folds it into M.
        absolute = 1.0 if precision == "fp8" else 2.0 * 2.0 ** -4
        Aa = Aa + absolute * Aa.max(axis=1, keepdims=True) / 229376.0 / u
        Ba = Ba + absolute * Ba.max(axis=0, keepdims=True) / 229376.0 / u
    M = oracle.block_product(Aa, Ba, b, d["keep"])
    stride = osk.block_stride_prec(b, precision)
    g = K * stride * 2.0 ** -24 + (2.0 ** -14 if fp8 else 0.0)
    bound = ((1 + u) ** 2 - 1 + g) * M
    err = np.abs(C - ref)
    worst = np.max(err / bound)
    assert worst <= 1.0, (precision, worst)
    # relative Frobenius against the oracle on the same S, per precision
    rel = oracle.rel_frob(C, ref)
    limit = {"fp32": 1e-5, "bf16": 2e-2, "bf16x3": 1e-4, "fp8": 2e-1, "fp8x3": 2e-2}[precision]
    assert rel <= limit, (precision, rel)


def test_lognormal_split_forms_recover_accuracy(lognormal_case):
    c, d = LOGNORMAL_CASE, lognormal_case
    Ad, Bd = torch.from_numpy(d["A"]).cuda(), torch.from_numpy(d["B"]).cuda()
    err = {}
    for prec in ("bf16", "bf16x3", "fp8", "fp8x3"):
        C = host(osk.matmul(Ad, Bd, c["b"], c["N"], c["e"], seed=d["seed"], keep=d["keep"],
                            precision=prec))
        err[prec] = oracle.rel_frob(C, d["ref"])
    assert err["bf16x3"] < err["bf16"] / 16
    assert err["fp8x3"] < err["fp8"] / 8
