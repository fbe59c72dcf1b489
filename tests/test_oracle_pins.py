"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-types an oracle formula: each compares the oracle with
a value printed in the paper, a published generator's output, an exact
enumeration, a closed form derived from Lemma 1, a special case that reduces
to an ordinary matrix product, or a statistical property with a bound.
"""
import itertools
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Hash: SplitMix64 reading of the random choices
# ---------------------------------------------------------------------------

def test_splitmix64_published_stream():
    # First three outputs of SplitMix64 seeded with 0, as produced by the
    # public-domain reference generator (Steele, Lea & Flood 2014; the
    # splitmix64.c of Vigna): widely reproduced test values.
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [oracle.splitmix64_nth(0, j) for j in range(3)] == expect


def test_hash_counter_layout():
    # block index lives above bit 40 of the counter, the column index below.
    assert oracle.hash_word(7, 0, 5) == oracle.splitmix64_nth(7, 5)
    assert oracle.hash_word(7, 3, 5) == oracle.splitmix64_nth(7, (3 << 40) | 5)


@pytest.mark.parametrize("b", [256, 1000, 7])
def test_hash_buckets_uniform(b):
    # Algorithm "Calculating Count-sketch": buckets uniform on [1, b].
    n = 1 << 16
    h, _ = oracle.hash_tables(1234, 3, n, b)
    assert h.min() >= 0 and h.max() < b
    for blk in range(3):
        counts = np.bincount(h[blk], minlength=b)
        chi2 = float(np.sum((counts - n / b) ** 2 / (n / b)))
        assert stats.chi2.sf(chi2, b - 1) > 1e-4, (blk, chi2)


def test_hash_signs_fair():
    # Algorithm "Calculating Count-sketch": each sign -1 with probability 1/2.
    n = 1 << 16
    _, s = oracle.hash_tables(99, 4, n, 64)
    for blk in range(4):
        mean = float(s[blk].astype(np.float64).mean())
        assert abs(mean) < 5.0 / np.sqrt(n)


def test_hash_blocks_independent():
    # Lemma 2 needs independent blocks: cross-block bucket collisions occur at
    # rate 1/b and signs agree at rate 1/2.
    n, b = 1 << 16, 64
    h, s = oracle.hash_tables(5, 2, n, b)
    p = 1.0 / b
    rate = float(np.mean(h[0] == h[1]))
    assert abs(rate - p) < 5 * np.sqrt(p * (1 - p) / n)
    agree = float(np.mean(s[0] == s[1]))
    assert abs(agree - 0.5) < 5 * np.sqrt(0.25 / n)
    # the bucket and sign of one (block, index) are independent too
    rate_pos = float(np.mean(h[0][s[0] > 0] < b // 2))
    assert abs(rate_pos - 0.5) < 5 * np.sqrt(0.25 / (n / 2))


def test_hash_depends_on_seed():
    h0, s0 = oracle.hash_tables(1, 1, 4096, 128)
    h1, s1 = oracle.hash_tables(2, 1, 4096, 128)
    assert np.mean(h0 == h1) < 0.05


# ---------------------------------------------------------------------------
# The paper's worked example (Section 4.1, Eq. (count_sketch_example))
# ---------------------------------------------------------------------------

def _load_example():
    sections, cur = {}, None
    with open(os.path.join(GOLDEN, "count_sketch_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                sections[cur] = []
            else:
                sections[cur].append(line)
    ST = np.array([[float(v) for v in row.split()] for row in sections["printed_ST"]])
    buckets = {}
    for row in sections["buckets"]:
        key, cols = row.split(":")
        buckets[int(key)] = [int(c) for c in cols.split()]
    strag = {}
    for row in sections["straggler"]:
        key, cols = row.split(":")
        strag[int(key)] = [int(c) for c in cols.split()]
    return ST, buckets, strag


def _example_tables():
    ST, buckets, _ = _load_example()
    n, b = ST.shape[1], ST.shape[0]
    h = np.full((1, n), -1, dtype=np.int32)
    for bucket, cols in buckets.items():
        for c in cols:
            h[0, c - 1] = bucket - 1          # 1-based in the paper, 0-based here
    assert np.all(h >= 0)
    sigma = np.array([[int(ST[h[0, k], k]) for k in range(n)]], dtype=np.int8)
    return ST, h, sigma, b


def test_example_prose_matches_printed_matrix():
    ST, buckets, _ = _load_example()
    assert ST.shape == (3, 9)
    # every column of S_c^T holds exactly one +-1: one bucket, one sign
    assert np.all(np.sum(ST != 0, axis=0) == 1)
    assert set(np.unique(ST)) <= {-1.0, 0.0, 1.0}
    for bucket, cols in buckets.items():
        nz = sorted(int(c) + 1 for c in np.flatnonzero(ST[bucket - 1]))
        assert nz == sorted(cols)


def test_example_sketch_of_identity_is_printed_matrix():
    ST, h, sigma, b = _example_tables()
    I = np.eye(9)
    np.testing.assert_array_equal(oracle.sketch_cols(I, h, sigma, b), ST.T)
    np.testing.assert_array_equal(oracle.sketch_rows(I, h, sigma, b), ST)


def test_example_sketch_equals_product_with_printed_matrix():
    ST, h, sigma, b = _example_tables()
    rng = np.random.default_rng(3)
    A = rng.standard_normal((5, 9))
    B = rng.standard_normal((9, 4))
    np.testing.assert_allclose(oracle.sketch_cols(A, h, sigma, b), A @ ST.T, rtol=0, atol=1e-14)
    np.testing.assert_allclose(oracle.sketch_rows(B, h, sigma, b), ST @ B, rtol=0, atol=1e-14)


def test_example_straggler_loses_exactly_its_columns():
    # Losing output column 3 of the sketch discards input columns 3, 8, 9 and
    # nothing else.
    _, _, strag = _load_example()
    _, h, sigma, b = _example_tables()
    lost = [c - 1 for c in strag[3]]
    rng = np.random.default_rng(4)
    A = rng.standard_normal((6, 9))
    A2 = A.copy()
    A2[:, lost] = rng.standard_normal((6, len(lost)))   # change only the lost columns
    S1 = oracle.sketch_cols(A, h, sigma, b)
    S2 = oracle.sketch_cols(A2, h, sigma, b)
    np.testing.assert_array_equal(S1[:, :2], S2[:, :2])  # buckets 1 and 2 unaffected
    assert np.all(S1[:, 2] != S2[:, 2])
    A3 = A.copy()
    keep_cols = [k for k in range(9) if k not in lost]
    A3[:, keep_cols] = 0.0
    assert np.all(oracle.sketch_cols(A3, h, sigma, b)[:, :2] == 0.0)


# ---------------------------------------------------------------------------
# Sketch as a matrix (Eq. (sketch_matrix)); special cases of the product
# ---------------------------------------------------------------------------

def test_sketch_of_identity_is_the_sketch_matrix():
    n, b, nblk = 50, 8, 3
    h, s = oracle.hash_tables(11, nblk, n, b)
    S = oracle.literal_blocks(h, s, b)
    # each row of every block holds one +-1
    assert np.all(np.sum(S != 0, axis=1) == nblk)
    np.testing.assert_array_equal(oracle.sketch_cols(np.eye(n), h, s, b), S)
    np.testing.assert_array_equal(oracle.sketch_rows(np.eye(n), h, s, b), S.T)


def test_sketch_is_linear():
    n, b, nblk = 40, 8, 2
    h, s = oracle.hash_tables(12, nblk, n, b)
    rng = np.random.default_rng(5)
    X, Y = rng.standard_normal((7, n)), rng.standard_normal((7, n))
    lhs = oracle.sketch_cols(2.0 * X - 3.0 * Y, h, s, b)
    rhs = 2.0 * oracle.sketch_cols(X, h, s, b) - 3.0 * oracle.sketch_cols(Y, h, s, b)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)
    P, Q = rng.standard_normal((n, 5)), rng.standard_normal((n, 5))
    lhs = oracle.sketch_rows(P + 0.5 * Q, h, s, b)
    rhs = oracle.sketch_rows(P, h, s, b) + 0.5 * oracle.sketch_rows(Q, h, s, b)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)


@pytest.mark.parametrize("N,e", [(1, 0), (3, 1)])
def test_exact_product_when_blocks_are_signed_permutations(N, e):
    # b = n and every h_i a permutation: S_i S_i^T = I, so C = AB exactly.
    m, n, l = 9, 32, 7
    rng = np.random.default_rng(6)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    h = np.stack([rng.permutation(n) for _ in range(N + e)]).astype(np.int32)
    s = rng.choice(np.array([-1, 1], dtype=np.int8), size=(N + e, n))
    keep = oracle.default_keep(N, e)
    C = oracle.sketched_matmul(A, B, n, N, e, keep=keep, h=h, sigma=s)
    np.testing.assert_allclose(C, A @ B, rtol=1e-12, atol=1e-12)


def test_b_one_gives_rank_one_sum():
    # b = 1: every index shares bucket 0, so A S_i = A sigma_i and
    # S_i^T B = sigma_i^T B, and C = (1/K) sum_i (A sigma_i)(sigma_i^T B).
    m, n, l, N, e = 6, 20, 5, 3, 1
    rng = np.random.default_rng(7)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    h, s = oracle.hash_tables(21, N + e, n, 1)
    assert np.all(h == 0)
    keep = synthetic.random_keep(N, e, 3)
    C = oracle.sketched_matmul(A, B, 1, N, e, keep=keep, h=h, sigma=s)
    ref = np.zeros((m, l))
    for i in np.flatnonzero(keep):
        sv = s[i].astype(np.float64)
        ref += np.outer(A @ sv, sv @ B)
    ref /= keep.sum()
    np.testing.assert_allclose(C, ref, rtol=1e-12, atol=1e-12)


def test_product_is_mean_of_single_block_products():
    m, n, l, b, N, e = 8, 64, 6, 8, 3, 2
    rng = np.random.default_rng(8)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    h, s = oracle.hash_tables(31, N + e, n, b)
    keep = np.array([1, 0, 1, 1, 0], dtype=np.uint8)
    C = oracle.sketched_matmul(A, B, b, N, e, keep=keep, h=h, sigma=s)
    parts = []
    for i in np.flatnonzero(keep):
        one = np.zeros(N + e, dtype=np.uint8)
        one[i] = 1
        parts.append(oracle.sketched_matmul(A, B, b, N, e, keep=one, h=h, sigma=s))
    np.testing.assert_allclose(C, np.mean(parts, axis=0), rtol=1e-12, atol=1e-12)


def test_oracle_matches_literal_dense_definition():
    m, n, l, b, N, e = 10, 60, 7, 8, 4, 1
    rng = np.random.default_rng(9)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    h, s = oracle.hash_tables(41, N + e, n, b)
    keep = synthetic.random_keep(N, e, 41)
    assert keep.sum() == N
    C = oracle.sketched_matmul(A, B, b, N, e, keep=keep, h=h, sigma=s)
    L = oracle.literal_product(A, B, h, s, b, N, keep)
    np.testing.assert_allclose(C, L, rtol=1e-12, atol=1e-12)


def test_sampled_entries_agree_with_full_product():
    m, n, l, b, N, e = 12, 80, 9, 16, 3, 1
    A, B = synthetic.gaussian_pair(m, n, l, 2, dtype=np.float32)
    keep = synthetic.random_keep(N, e, 2)
    C = oracle.sketched_matmul(A, B, b, N, e, seed=2, keep=keep)
    rows = np.array([0, 3, 11, 5, 5])
    cols = np.array([0, 8, 2, 2, 7])
    v = oracle.sampled_entries(A, B, rows, cols, b, N, e, seed=2, keep=keep)
    np.testing.assert_allclose(v, C[rows, cols], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Lemma 1 / Lemma 2 by exhaustive enumeration of every sketch
# ---------------------------------------------------------------------------

def _all_single_block_tables(n, b):
    hs, ss = [], []
    for hv in itertools.product(range(b), repeat=n):
        for sv in itertools.product((-1, 1), repeat=n):
            hs.append(hv)
            ss.append(sv)
    return np.array(hs, dtype=np.int32), np.array(ss, dtype=np.int8)


def _lemma1_variance(x, y, b):
    # Lemma 1: Var = (1/b) (sum_{j != l} x_j^2 y_l^2 + sum_{j != l} x_j y_j x_l y_l)
    n = len(x)
    t1 = sum(x[j] ** 2 * y[l] ** 2 for j in range(n) for l in range(n) if j != l)
    t2 = sum(x[j] * y[j] * x[l] * y[l] for j in range(n) for l in range(n) if j != l)
    return (t1 + t2) / b


@pytest.mark.parametrize("n,b", [(4, 2), (5, 3), (3, 4)])
def test_lemma1_exact_mean_and_variance(n, b):
    rng = np.random.default_rng(10 + n)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    h, s = _all_single_block_tables(n, b)
    cnt = h.shape[0]
    xa = oracle.sketch_cols(x[None, :], h, s, b).reshape(cnt, b)
    yb = oracle.sketch_rows(y[:, None], h, s, b).reshape(cnt, b)
    v = np.sum(xa * yb, axis=1)                     # x^T S_c S_c^T y per sketch
    assert abs(v.mean() - x @ y) < 1e-12 * (1 + abs(x @ y))
    var = float(np.mean((v - x @ y) ** 2))
    assert var == pytest.approx(_lemma1_variance(x, y, b), rel=1e-10)
    # and the two upper bounds stated with it
    assert var <= ((x @ y) ** 2 + (x @ x) * (y @ y)) / b + 1e-12
    assert var <= 2.0 / b * (x @ x) * (y @ y) + 1e-12


def test_lemma2_exact_mean_and_variance_two_blocks():
    # S = N^{-1/2}(S_1, S_2) with independent blocks: mean x^T y, variance
    # Var_1 / N, within the 2/d bound (d = N b).
    n, b, N = 3, 2, 2
    rng = np.random.default_rng(20)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    h1, s1 = _all_single_block_tables(n, b)
    vals = []
    for i in range(h1.shape[0]):
        for j in range(h1.shape[0]):
            h = np.stack([h1[i], h1[j]])
            s = np.stack([s1[i], s1[j]])
            vals.append(oracle.sketched_matmul(x[None, :], y[:, None], b, N, 0, h=h, sigma=s)[0, 0])
    vals = np.array(vals)
    assert abs(vals.mean() - x @ y) < 1e-12
    var = float(np.mean((vals - x @ y) ** 2))
    assert var == pytest.approx(_lemma1_variance(x, y, b) / N, rel=1e-10)
    assert var <= 2.0 / (N * b) * (x @ x) * (y @ y)


def _second_moment_closed_form(A, B, b, K):
    """E||A S S^T B - AB||_F^2 for K kept independent count-sketch blocks of
    width b (sum of Lemma 1's variance over all entries of AB, divided by K):
    (||A||^2 ||B||^2 + ||AB||^2 - 2 sum_k ||A[:,k]||^2 ||B[k,:]||^2) / (K b)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    AB = A @ B
    cross = float(np.sum(np.sum(A * A, axis=0) * np.sum(B * B, axis=1)))
    return (oracle.frob2(A) * oracle.frob2(B) + oracle.frob2(AB) - 2.0 * cross) / (K * b)


def test_second_moment_exact_enumeration():
    m, n, l, b = 3, 3, 2, 2
    rng = np.random.default_rng(21)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    AB = A @ B
    h1, s1 = _all_single_block_tables(n, b)
    errs = []
    for i in range(h1.shape[0]):
        C = oracle.sketched_matmul(A, B, b, 1, 0, h=h1[i:i + 1], sigma=s1[i:i + 1])
        errs.append(oracle.frob2(C - AB))
    assert float(np.mean(errs)) == pytest.approx(_second_moment_closed_form(A, B, b, 1), rel=1e-10)


# ---------------------------------------------------------------------------
# Statistical behaviour over hash seeds (Lemma 2, Lemma 3, main theorem)
# ---------------------------------------------------------------------------

def _seed_runs(A, B, b, N, e, T, keep=None, seed0=1000):
    return [oracle.sketched_matmul(A, B, b, N, e, seed=seed0 + t, keep=keep) for t in range(T)]


def test_second_moment_monte_carlo_matches_closed_form():
    m, n, l, b, N, e = 8, 64, 6, 4, 2, 1
    rng = np.random.default_rng(22)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    keep = oracle.default_keep(N, e)
    Cs = _seed_runs(A, B, b, N, e, 600, keep=keep)
    AB = A @ B
    mc = float(np.mean([oracle.frob2(C - AB) for C in Cs]))
    assert mc == pytest.approx(_second_moment_closed_form(A, B, b, N), rel=0.12)


def test_unbiased_mean_over_seeds():
    # Lemma 2: E[A S S^T B] = AB; E||mean_T - AB||^2 = E1 / T exactly.
    m, n, l, b, N, e = 8, 64, 6, 4, 2, 1
    rng = np.random.default_rng(23)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    T = 400
    Cs = _seed_runs(A, B, b, N, e, T, keep=oracle.default_keep(N, e))
    E1 = _second_moment_closed_form(A, B, b, N)
    dev = oracle.frob2(np.mean(Cs, axis=0) - A @ B)
    assert dev <= 3.0 * E1 / T


def test_extra_kept_blocks_need_one_over_k():
    # K = N + e kept blocks: weight 1/K keeps the product unbiased; weight 1/N
    # would inflate it by K/N, which this check would see.
    m, n, l, b, N, e = 8, 64, 6, 4, 2, 1
    rng = np.random.default_rng(24)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    T = 400
    keep = np.ones(N + e, dtype=np.uint8)
    Cs = _seed_runs(A, B, b, N, e, T, keep=keep)
    AB = A @ B
    E1 = _second_moment_closed_form(A, B, b, N + e)
    mean = np.mean(Cs, axis=0)
    assert oracle.frob2(mean - AB) <= 3.0 * E1 / T
    wrong = mean * (N + e) / N
    assert oracle.frob2(wrong - AB) > 10.0 * E1 / T


def test_lemma3_bound_holds():
    # E||AB - A S S^T B||^2 <= (2/d) ||A||^2 ||B||^2, d = N b.
    m, n, l, b, N, e = 10, 128, 8, 8, 3, 1
    rng = np.random.default_rng(25)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    bound = 2.0 / (N * b) * oracle.frob2(A) * oracle.frob2(B)
    assert _second_moment_closed_form(A, B, b, N) <= bound
    Cs = _seed_runs(A, B, b, N, e, 200, keep=oracle.default_keep(N, e))
    mc = float(np.mean([oracle.frob2(C - A @ B) for C in Cs]))
    assert mc <= bound


def test_main_theorem_tail():
    # d = 2/(eps theta) gives P(err^2 > eps ||A||^2 ||B||^2) <= theta, with e
    # blocks ignored.
    m, n, l, b, N, e = 12, 200, 10, 8, 4, 2
    d = N * b
    theta = 0.25
    eps = 2.0 / (d * theta)
    rng = np.random.default_rng(26)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    T = 300
    thr = eps * oracle.frob2(A) * oracle.frob2(B)
    AB = A @ B
    exceed = 0
    for t in range(T):
        keep = synthetic.random_keep(N, e, 500 + t)
        C = oracle.sketched_matmul(A, B, b, N, e, seed=500 + t, keep=keep)
        exceed += oracle.frob2(C - AB) > thr
    assert exceed / T <= theta + 3 * np.sqrt(theta * (1 - theta) / T)


def test_rank_refined_bound():
    # Section 4, after the main theorem: for rank(A) = r,
    # ||A||_2 <= ||A||_F <= sqrt(r) ||A||_2, so d = 2/(eps theta) gives
    # P(err^2 > eps r ||A||_2^2 ||B||_F^2) <= theta, and a sketch r times
    # wider, z = r (d + e b), gives P(err^2 > eps ||A||_2^2 ||B||_F^2) <= theta.
    m, n, l, r, b, N, e = 16, 256, 10, 4, 8, 4, 1
    rng = np.random.default_rng(31)
    # a fat rank-r A with equal singular values (||A||_F^2 = r ||A||_2^2)
    Q1, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, r)))
    A = 3.0 * Q1 @ Q2.T
    B = rng.standard_normal((n, l))
    s2 = np.linalg.norm(A, 2) ** 2
    fa = oracle.frob2(A)
    assert np.linalg.matrix_rank(A) == r
    assert s2 <= fa + 1e-9 and fa <= r * s2 * (1 + 1e-12)
    assert fa == pytest.approx(r * s2, rel=1e-12)
    d = N * b
    theta = 0.25
    eps = 2.0 / (d * theta)
    AB = A @ B
    fb = oracle.frob2(B)
    T = 200
    slack = 3 * np.sqrt(theta * (1 - theta) / T)
    base, wide, wide_mean = 0, 0, 0.0
    for t in range(T):
        seed = 900 + t
        keep = synthetic.random_keep(N, e, seed)
        C = oracle.sketched_matmul(A, B, b, N, e, seed=seed, keep=keep)
        base += oracle.frob2(C - AB) > eps * r * s2 * fb
        keep_w = synthetic.random_keep(r * N, r * e, seed)
        Cw = oracle.sketched_matmul(A, B, b, r * N, r * e, seed=seed, keep=keep_w)
        ew = oracle.frob2(Cw - AB)
        wide += ew > eps * s2 * fb
        wide_mean += ew / T
    assert base / T <= theta + slack
    assert wide / T <= theta + slack
    # the wider sketch's mean error is the closed form at K = r N (so the
    # threshold above is eps theta / (its mean) away, not vacuous)
    assert wide_mean == pytest.approx(_second_moment_closed_form(A, B, b, r * N), rel=0.2)
    assert wide_mean <= eps * theta * s2 * fb


def test_graceful_degradation_more_losses_more_error():
    # Dropping more blocks than provisioned still gives an unbiased product
    # with larger error (section 4.1, "graceful degradation").
    m, n, l, b, N, e = 8, 128, 6, 8, 4, 0
    rng = np.random.default_rng(27)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    AB = A @ B
    err = {}
    for K in (4, 2, 1):
        keep = np.zeros(N, dtype=np.uint8)
        keep[:K] = 1
        errs = [oracle.frob2(oracle.sketched_matmul(A, B, b, N, e, seed=700 + t, keep=keep) - AB)
                for t in range(150)]
        err[K] = float(np.mean(errs))
        assert err[K] == pytest.approx(_second_moment_closed_form(A, B, b, K), rel=0.25)
    assert err[4] < err[2] < err[1]


def test_config1_error_level():
    # 256x4096 by 4096x256 Gaussian, b=256, N=4, e=1 with one random block
    # dropped: one instance's error sits near the closed-form expectation.
    m, n, l, b, N, e, seed = 256, 4096, 256, 256, 4, 1, 1
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    keep = synthetic.random_keep(N, e, seed)
    C = oracle.sketched_matmul(A, B, b, N, e, seed=seed, keep=keep)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    AB = A64 @ B64
    err2 = oracle.frob2(C - AB)
    expect = _second_moment_closed_form(A64, B64, b, N)
    assert err2 == pytest.approx(expect, rel=0.2)
    assert err2 <= 2.0 / (N * b) * oracle.frob2(A64) * oracle.frob2(B64)


# ---------------------------------------------------------------------------
# BF16 rounding (operands of the reduced-precision block product)
# ---------------------------------------------------------------------------

def _bf16_nearest_brute(x):
    """Nearest BF16 value to each FP32 x by enumeration of the two BF16
    neighbours (truncation and the next BF16 away from zero), ties to the
    one with an even last kept bit: the definition, written without the
    add-and-shift trick."""
    out = np.empty_like(x)
    for i, v in enumerate(x):
        bits = int(np.float32(v).view(np.uint32))
        lo_bits = bits & 0xFFFF0000
        hi_bits = lo_bits + 0x10000
        lo = np.uint32(lo_bits).view(np.float32)
        hi = np.uint32(hi_bits & 0xFFFFFFFF).view(np.float32)
        dlo = abs(float(v) - float(lo))
        dhi = abs(float(v) - float(hi)) if np.isfinite(hi) else np.inf
        if dlo < dhi:
            out[i] = lo
        elif dhi < dlo:
            out[i] = hi
        else:
            out[i] = lo if ((lo_bits >> 16) & 1) == 0 else hi
    return out


def test_bf16_round_worked_values():
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                      # halfway, 1.0 has an even last bit
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,      # halfway, rounds up to the even neighbour
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,   # above halfway
        -(one + 2.0 ** -8 + 2.0 ** -20): -(one + 2.0 ** -7),
        float(np.finfo(np.float32).max): np.inf,   # past the largest BF16 + half an ulp
        3.0e38: float(np.uint32(0x7F62 << 16).view(np.float32)),
        0.0: 0.0,
        2.0 ** -133: 2.0 ** -133,                  # a subnormal that is already BF16
    }
    x = np.array(list(cases), dtype=np.float32)
    want = np.array(list(cases.values()), dtype=np.float32)
    np.testing.assert_array_equal(oracle.bf16_round(x), want)
    assert np.isnan(oracle.bf16_round(np.array([np.nan], np.float32)))[0]


def test_bf16_round_matches_nearest_value_definition():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(3000).astype(np.float32),
                        (rng.standard_normal(2000) * 1e-39).astype(np.float32),  # subnormals
                        np.float32(1.0) + rng.integers(0, 1 << 16, 2000).astype(np.float32)
                        * np.float32(2.0 ** -23)])
    np.testing.assert_array_equal(oracle.bf16_round(x), _bf16_nearest_brute(x))


def test_bf16_split_recovers_sixteen_bits():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(10000).astype(np.float32)
    hi, lo = oracle.bf16_split(x)
    # BF16 keeps 8 significant bits: round to nearest is within 2^-8
    # relatively, so hi + lo leaves one BF16 rounding of the residual:
    # |x - hi - lo| <= 2^-8 |x - hi| <= 2^-16 |x| (normal range)
    assert np.all(oracle.bf16_round(hi) == hi) and np.all(oracle.bf16_round(lo) == lo)
    xd = np.abs(x.astype(np.float64))
    assert np.all(np.abs(x.astype(np.float64) - hi) <= 2.0 ** -8 * xd)
    r = np.abs(x.astype(np.float64) - hi - lo)
    assert np.all(r <= 2.0 ** -16 * xd)
    # and the split is not vacuous: the residual term matters
    assert np.mean(np.abs(x.astype(np.float64) - hi)) > 100 * np.mean(r)


# ---------------------------------------------------------------------------
# FP8 E4M3 with power-of-two block scales
# ---------------------------------------------------------------------------

def test_e4m3_value_table():
    v = oracle.e4m3_values()
    assert v[0] == 0 and v[1] == 2.0 ** -9 and v[7] == 7 * 2.0 ** -9
    assert v[8] == 2.0 ** -6                 # smallest normal continues the subnormals
    assert v[0x38] == 1.0 and v[126] == 448.0
    assert np.all(np.diff(v) > 0)            # codes are ordered by magnitude


def test_e4m3_round_worked_values():
    y = np.array([1.0, 1 + 1 / 16, 1 + 3 / 16, 1 + 1 / 16 + 1e-6, 448.0, -0.5625,
                  2.0 ** -10, 3 * 2.0 ** -10, 2.0 ** -10 + 1e-9, 0.0])
    want = np.array([1.0, 1.0, 1.25, 1.125, 448.0, -0.5625,
                     0.0, 2 * 2.0 ** -9, 2.0 ** -9, 0.0])
    np.testing.assert_array_equal(oracle.e4m3_round(y), want)
    v = oracle.e4m3_values()
    np.testing.assert_array_equal(oracle.e4m3_round(v), v)       # exact values stay
    np.testing.assert_array_equal(oracle.e4m3_round(-v), -v)


def test_e4m3_round_is_nearest():
    rng = np.random.default_rng(3)
    y = rng.uniform(-448, 448, 20000) * np.exp(rng.uniform(-14, 0, 20000))
    q = oracle.e4m3_round(y)
    v = oracle.e4m3_values()
    best = np.min(np.abs(np.abs(y)[:, None] - v[None, :]), axis=1)
    np.testing.assert_array_equal(np.abs(np.abs(y) - np.abs(q)), best)


def test_e8m0_scale_exponent():
    assert oracle.e8m0_scale_exponent(448.0) == 0
    assert oracle.e8m0_scale_exponent(449.0) == 1
    assert oracle.e8m0_scale_exponent(896.0) == 1
    assert oracle.e8m0_scale_exponent(897.0) == 2
    assert oracle.e8m0_scale_exponent(1.0) == -8        # 448 * 2^-8 = 1.75 >= 1 > 0.875
    assert oracle.e8m0_scale_exponent(0.0) == -127
    assert oracle.e8m0_scale_exponent(1e-45) == -127


def test_fp8_block_quantize_error_bound():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((16, 256)) * np.exp(rng.standard_normal((16, 1)) * 3)
    q, s = oracle.fp8_block_quantize(x)
    assert s.shape == (16, 8)
    blockmax = np.repeat(np.abs(x).reshape(16, 8, 32).max(axis=2), 32, axis=1)
    # normal range: 3 fraction bits (2^-4 relative); below it the step is
    # 2^(s-9) < blockmax / 224 / 512 -> half a step
    assert np.all(np.abs(x - q) <= 2.0 ** -4 * np.abs(x) + blockmax / 224 / 1024 + 1e-300)
    assert np.all(np.abs(q) <= 448.0 * np.repeat(np.ldexp(1.0, s), 32, axis=1))
    hi, lo = oracle.fp8_split(x)
    assert np.array_equal(hi, q)
    assert np.mean(np.abs(x - hi - lo)) < np.mean(np.abs(x - hi)) / 8


# ---------------------------------------------------------------------------
# Sketched Hessian / Gram matrix (Section 5.2, Eq. (int_point) and the
# Hessian after it): H = (1/K) sum_i (A D^{1/2} S_i)(A D^{1/2} S_i)^T
# ---------------------------------------------------------------------------

def _log_uniform(rng, n, lo=1e-6, hi=1e6):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


@pytest.mark.parametrize("N,e", [(1, 0), (2, 1)])
def test_gram_with_permutation_sketch_is_the_hessian(N, e):
    # b = n and permutations h_i: S_i S_i^T = I, so H = A D A^T exactly (the
    # weights enter as D, i.e. D^{1/2} on each side).
    m, n = 7, 24
    rng = np.random.default_rng(40)
    A = rng.standard_normal((m, n))
    d = _log_uniform(rng, n)
    h = np.stack([rng.permutation(n) for _ in range(N + e)]).astype(np.int32)
    s = rng.choice(np.array([-1, 1], dtype=np.int8), size=(N + e, n))
    H = oracle.sketched_gram(A, d, n, N, e, keep=oracle.default_keep(N, e), h=h, sigma=s)
    ref = (A * d[None, :]) @ A.T
    np.testing.assert_allclose(H, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_gram_zero_weights_remove_their_indices():
    # d_k = 0 removes index k from the sum: equal to the problem without
    # those columns (and without their bucket/sign entries), bit for bit.
    m, n, b, N, e = 5, 40, 6, 3, 1
    rng = np.random.default_rng(41)
    A = rng.standard_normal((m, n))
    d = _log_uniform(rng, n)
    drop = np.zeros(n, bool)
    drop[rng.choice(n, 13, replace=False)] = True
    d0 = d.copy()
    d0[drop] = 0.0
    h, s = oracle.hash_tables(77, N + e, n, b)
    keep = synthetic.random_keep(N, e, 5)
    H = oracle.sketched_gram(A, d0, b, N, e, keep=keep, h=h, sigma=s)
    Hr = oracle.sketched_gram(A[:, ~drop], d[~drop], b, N, e, keep=keep,
                              h=np.ascontiguousarray(h[:, ~drop]),
                              sigma=np.ascontiguousarray(s[:, ~drop]))
    assert np.array_equal(H, Hr)


def test_gram_brute_force_dense_sketch():
    # tiny case against the dense definition with S = N^{-1/2}(S_1 .. S_{N+e})
    m, n, b, N, e = 4, 11, 3, 2, 1
    rng = np.random.default_rng(42)
    A = rng.standard_normal((m, n))
    d = _log_uniform(rng, n, 1e-2, 1e2)
    h, s = oracle.hash_tables(9, N + e, n, b)
    keep = np.array([1, 0, 1], np.uint8)
    H = oracle.sketched_gram(A, d, b, N, e, keep=keep, h=h, sigma=s)
    W = A * np.sqrt(d)[None, :]
    S = np.zeros((n, (N + e) * b))
    for i in range(N + e):
        for k in range(n):
            S[k, i * b + h[i, k]] = s[i, k]
    cols = [i * b + c for i in range(N + e) if keep[i] for c in range(b)]
    SK = S[:, cols]
    ref = (W @ SK) @ (W @ SK).T / keep.sum()
    np.testing.assert_allclose(H, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_gram_is_symmetric_psd_and_unbiased():
    # symmetric positive semidefinite for every draw; its mean over
    # independent hash seeds tends to A D A^T (E[S_i S_i^T] = I), within a
    # few standard errors of the empirical spread.
    m, n, b, N, e, T = 5, 48, 8, 2, 0, 400
    rng = np.random.default_rng(43)
    A = rng.standard_normal((m, n))
    d = _log_uniform(rng, n, 1e-1, 1e1)
    ref = (A * d[None, :]) @ A.T
    Hs = np.stack([oracle.sketched_gram(A, d, b, N, e, seed=1000 + t) for t in range(T)])
    for H in Hs[:20]:
        assert np.array_equal(H, H.T)
        assert np.linalg.eigvalsh(H).min() >= -1e-9 * np.abs(H).max()
    mean = Hs.mean(axis=0)
    se = Hs.std(axis=0, ddof=1) / np.sqrt(T)
    z = np.abs(mean - ref) / np.maximum(se, 1e-12)
    assert z.max() < 5.0, z.max()
    # a missing square root (A D^2 A^T) or a missing 1/K would be far off
    assert oracle.rel_frob(mean, ref) < 0.1


# ---------------------------------------------------------------------------
# Per-C-block keep masks (Algorithm "OverSketch": every b x b block of C has
# its own stragglers)
# ---------------------------------------------------------------------------

def test_cmask_uniform_mask_is_the_global_product():
    m, n, l, b, N, e = 13, 40, 11, 5, 3, 1
    rng = np.random.default_rng(50)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    keep = np.array([1, 0, 1, 1], np.uint8)
    cm = np.broadcast_to(keep, (-(-m // b), -(-l // b), N + e)).copy()
    C = oracle.sketched_matmul_cmask(A, B, b, N, e, cm, seed=3)
    assert np.array_equal(C, oracle.sketched_matmul(A, B, b, N, e, seed=3, keep=keep))


def test_cmask_blocks_follow_the_dense_definition():
    # each C block against A_I S_K S_K^T B_J with its own kept set, dense S
    # (S = N^{-1/2}[S_1 ..], so the 1/N factor is traded for 1/K_IJ); blocks
    # that keep nothing are zero
    m, n, l, b, N, e = 7, 17, 9, 3, 2, 2
    rng = np.random.default_rng(51)
    A, B = rng.standard_normal((m, n)), rng.standard_normal((n, l))
    h, s = oracle.hash_tables(8, N + e, n, b)
    nbI, nbJ = -(-m // b), -(-l // b)
    cm = (rng.random((nbI, nbJ, N + e)) < 0.5).astype(np.uint8)
    cm[0, 0] = 0
    cm[1, 1] = [1, 0, 0, 0]
    cm[-1, -1] = 1
    C = oracle.sketched_matmul_cmask(A, B, b, N, e, cm, h=h, sigma=s)
    for I in range(nbI):
        for J in range(nbJ):
            r = slice(I * b, min(m, (I + 1) * b))
            c = slice(J * b, min(l, (J + 1) * b))
            K = int(cm[I, J].sum())
            if K == 0:
                assert np.all(C[r, c] == 0)
                continue
            ref = oracle.literal_product(A[r], B[:, c], h, s, b, N, cm[I, J]) * (N / K)
            np.testing.assert_allclose(C[r, c], ref, rtol=1e-12, atol=1e-12)
