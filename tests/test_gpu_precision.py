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
