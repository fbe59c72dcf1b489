"""The paper's constant-matrix workloads at the paper's own sizes, on one GPU
(the experiments of Section 5.1, Fig. 5b, and Section 5.3), with a keep mask
per b x b block of C as in those experiments (every block of C ignores its
own e workers).

  - Fig. 5b: A(x, y) = x + y, m = l = 10b, n = 60b, b = 2048, B = A^T,
    z = 30b, e = 4 workers ignored per block of C.  The paper prints a mean
    relative Frobenius error of 0.8 % over ten sketches; the paper's hash is
    unknown, so the printed value is an order-of-magnitude check: the mean
    over ten sketches must be <= 1 %.
  - Section 5.3: A(x, y) = x + y and B(x, y) = x y, n x n with n = 24000,
    b = 4000, z = n/2 + b (4 workers per block of C), one ignored per block:
    mean error over ten sketches under 2 % (the paper's statement).

Both also hold the mean over the ten sketches to within a factor 1.5 of the
RMS error that the second moment gives (Lemma 1's variance summed over the
entries of AB, over K).  For these rank-2 inputs a single sketch's error is
widely spread: a reduced-size Monte-Carlo of the Fig. 5b shape (b = 16 and
32, 200 sketches) put single errors between 0.37 and 1.56 times the RMS
(10th to 90th percentile) and means of ten between 0.60 and 1.29 times it.
Both compare sampled entries of the first sketch's C with the FP64 oracle
(per block of C, with that block's mask), relative error over the sample
<= 1e-5.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1811_02653_amd as osk  # noqa: E402

TOL = 1e-5


def _predicted(nA2, nB2, nAB2, cross, K, b):
    return ((nA2 * nB2 + nAB2 - 2.0 * cross) / (K * b) / nAB2) ** 0.5


def _sampled_parity(C, rows, cols, A_rows, B_cols, b, N, e, seed, cmask):
    """C[rows, cols] against the oracle, one call per block of C; A_rows(r)
    gives rows r of A and B_cols(c) columns c of B as FP64 host arrays."""
    got = C[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].double().cpu().numpy()
    ref = np.empty_like(got)
    n = A_rows(rows[:1]).shape[1]
    h, s = oracle.hash_tables(seed, N + e, n, b)
    blocks = {}
    for t, (r, c) in enumerate(zip(rows, cols)):
        blocks.setdefault((r // b, c // b), []).append(t)
    for (I, J), ts in blocks.items():
        ts = np.array(ts)
        ur, ir = np.unique(rows[ts], return_inverse=True)
        uc, ic = np.unique(cols[ts], return_inverse=True)
        ref[ts] = oracle.sampled_entries(A_rows(ur), B_cols(uc), ir, ic, b, N, e, h=h, sigma=s,
                                         keep=cmask[I, J])
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


def _sample(m, l, count, seed):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, m, count)
    cols = rng.integers(0, l, count)
    rows[:4], cols[:4] = [0, 0, m - 1, m - 1], [0, l - 1, 0, l - 1]
    return rows, cols


SKETCHES = 10


def test_fig5b_error_and_parity():
    b, nb, e, seed = 2048, 30, 4, 11
    m, n = 10 * b, 60 * b
    A, x, y = synthetic.paper_matrices_device(m, n)
    G, nA2, _, cross = synthetic.paper_exact_products(x, y)
    nG2 = torch.sum(G * G).item()
    C = torch.empty((m, m), dtype=torch.float32, device="cuda")
    errs = []
    for k in reversed(range(SKETCHES)):          # the first sketch last: C holds it
        cm = synthetic.random_cmask(m // b, m // b, nb - e, e, seed + k)
        osk.matmul_cmask(A, A.t(), b, nb - e, e, cm, seed=seed + k, out=C)
        torch.cuda.synchronize()
        errs.append((torch.sum((C.double() - G) ** 2).item() / nG2) ** 0.5)
    err = float(np.mean(errs))
    pred = _predicted(nA2, nA2, nG2, cross, nb - e, b)
    assert err <= 0.01, errs
    assert pred / 1.5 <= err <= 1.5 * pred, (errs, pred)
    del G
    xs = np.arange(1, m + 1, dtype=np.float64)
    ys = np.arange(1, n + 1, dtype=np.float64)
    A_rows = lambda r: xs[r][:, None] + ys[None, :]
    B_cols = lambda c: (xs[c][:, None] + ys[None, :]).T        # B = A^T
    rows, cols = _sample(m, m, 96, seed)
    assert _sampled_parity(C, rows, cols, A_rows, B_cols, b, nb - e, e, seed, cm) <= TOL   # k = 0


def test_section_5_3_error_and_parity():
    n, b, seed = 24000, 4000, 12
    nb = n // (2 * b) + 1                      # z = n/2 + b
    A, B, x, y, z = synthetic.paper_matrices_device(n, n, n)
    AB, nA2, nB2, cross = synthetic.paper_exact_products(x, y, z)
    nAB2 = torch.sum(AB * AB).item()
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    errs = []
    for k in reversed(range(SKETCHES)):          # the first sketch last: C holds it
        cm = synthetic.random_cmask(n // b, n // b, nb - 1, 1, seed + k)
        osk.matmul_cmask(A, B, b, nb - 1, 1, cm, seed=seed + k, out=C)
        torch.cuda.synchronize()
        errs.append((torch.sum((C.double() - AB) ** 2).item() / nAB2) ** 0.5)
    err = float(np.mean(errs))
    pred = _predicted(nA2, nB2, nAB2, cross, nb - 1, b)
    assert err < 0.02, errs
    assert pred / 1.5 <= err <= 1.5 * pred, (errs, pred)
    del AB
    ks = np.arange(1, n + 1, dtype=np.float64)
    A_rows = lambda r: ks[r][:, None] + ks[None, :]
    # the FP32-rounded x * y values the GPU was given, exactly
    B_cols = lambda c: (ks[:, None] * ks[c][None, :]).astype(np.float32).astype(np.float64)
    rows, cols = _sample(n, n, 96, seed)
    assert _sampled_parity(C, rows, cols, A_rows, B_cols, b, nb - 1, 1, seed, cm) <= TOL   # k = 0
