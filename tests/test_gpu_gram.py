"""GPU parity of the batched sketched Gram matrices (the Hessian sketch of the
interior-point method, Section 5.2) against the FP64 oracle, through the C ABI.

Each H_k is compared with oracle.sketched_gram on the same inputs and hash
seed: relative Frobenius error <= 1e-5 (FP32 sketch sums over about n/b
terms and an FP32 product over K*b terms, the same bound as the plain
product's parity tests).  Re-runs of the same plan (autotuned, reused
prepared sketches, graph replays) must reproduce the eager result bit for bit.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1811_02653_amd as osk  # noqa: E402

TOL = 1e-5


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _problems(specs, seed):
    """specs: (m, n, b, N, e, drop) per problem; A ~ N(0,1), d log-uniform
    in [1e-6, 1e6]."""
    rng = synthetic.data_rng(seed)
    out = []
    for t, (m, n, b, N, e, drop) in enumerate(specs):
        A = rng.standard_normal((m, n), dtype=np.float32)
        d = np.exp(rng.uniform(np.log(1e-6), np.log(1e6), size=n)).astype(np.float32)
        keep = synthetic.random_keep(N, e, seed + t, drop=drop)
        out.append((A, d, b, N, e, keep, seed * 100 + t))
    return out


def _batch(probs, **kw):
    return osk.GramBatch([dev(p[0]) for p in probs], [dev(p[1]) for p in probs],
                         b=[p[2] for p in probs], N=[p[3] for p in probs],
                         e=[p[4] for p in probs], keeps=[p[5] for p in probs],
                         seeds=[p[6] for p in probs], **kw)


def _oracle(p):
    A, d, b, N, e, keep, seed = p
    return oracle.sketched_gram(A, d, b, N, e, seed=seed, keep=keep)


SPECS = [
    (300, 6000, 150, 6, 1, 1),      # the batch workload's shape rules at small m
    (513, 2050, 64, 4, 2, 3),       # ragged tiles, K < N
    (1, 50, 1, 1, 0, 0),            # degenerate
    (130, 129, 200, 2, 1, 0),       # n < b, K > N
    (257, 5140, 129, 3, 0, 0),      # one row past a 256 tile
    (40, 800, 20, 6, 1, 1),
]


MIXED = osk.gram.MIXED
# side of the tiles whose upper triangle is written when full = 0
WRITTEN_SIDE = {256: 256, 128: 128, MIXED: 128}


@pytest.mark.parametrize("tile", [256, 128, MIXED])
@pytest.mark.parametrize("full", [True, False])
def test_gram_batch_vs_oracle(tile, full):
    probs = _problems(SPECS, 11)
    outs = [torch.full((p[0].shape[0], p[0].shape[0]), -7.0, device="cuda") for p in probs]
    gb = _batch(probs, full=full, out=outs, tile=tile)
    assert gb.config[0] == tile and gb.config[1] > 0
    Hs = [host(h) for h in gb.run()]
    for p, H in zip(probs, Hs):
        ref = _oracle(p)
        m = ref.shape[0]
        if full:
            assert oracle.rel_frob(H, ref) <= TOL, (m, oracle.rel_frob(H, ref))
            assert np.max(np.abs(H - H.T)) <= 1e-6 * np.abs(ref).max()
        else:
            # tiles on or above the diagonal are written, the others untouched
            side = WRITTEN_SIDE[tile]
            ti = np.arange(m)[:, None] // side
            tj = np.arange(m)[None, :] // side
            upper = ti <= tj
            assert np.all(H[~upper] == -7.0)
            assert oracle.rel_frob(np.where(upper, H, 0), np.where(upper, ref, 0)) <= TOL


# sizes around the 128 and 256 tile boundaries: a diagonal 256 tile of one,
# two or three 128 tiles, last tile columns of at most and of more than 128
# columns, an odd count of 128 tiles (one unpaired)
EDGE_M = [1, 100, 128, 129, 200, 255, 256, 257, 300, 383, 384, 385, 511, 512, 513, 640, 700]


@pytest.mark.parametrize("full", [True, False])
def test_gram_batch_mixed_tile_edges(full):
    specs = [(m, 64 * (1 + k % 3), 32, 2, 1, 1) for k, m in enumerate(EDGE_M)]
    probs = _problems(specs, 15)
    outs = [torch.full((p[0].shape[0], p[0].shape[0]), -7.0, device="cuda") for p in probs]
    gb = _batch(probs, full=full, out=outs, tile=MIXED)
    mixed = [host(h) for h in gb.run()]
    gb.configure(256)
    whole = [host(h.clone()) for h in gb.run()]
    gb.close()
    for p, H, W in zip(probs, mixed, whole):
        ref = _oracle(p)
        m = ref.shape[0]
        upper = (np.arange(m)[:, None] // 128) <= (np.arange(m)[None, :] // 128)
        if full:
            assert oracle.rel_frob(H, ref) <= TOL, (m, oracle.rel_frob(H, ref))
            assert np.array_equal(H, H.T), m
            # the same dot products in the same K order as the 256 form
            assert oracle.rel_frob(H, W) <= 1e-6, m
        else:
            assert np.all(H[~upper] == -7.0), m
            assert oracle.rel_frob(np.where(upper, H, 0), np.where(upper, ref, 0)) <= TOL, m


def test_gram_batch_unweighted_equals_sketched_product():
    # d = None (D = I): H = the OverSketch product of A with A^T
    rng = synthetic.data_rng(12)
    A = rng.standard_normal((200, 3000), dtype=np.float32)
    gb = osk.GramBatch([dev(A)], None, b=100, N=4, e=1, seeds=[5])
    H = host(gb.run()[0])
    ref = oracle.sketched_matmul(A, A.T, 100, 4, 1, seed=5)
    assert oracle.rel_frob(H, ref) <= TOL


def test_gram_batch_permutation_sketch_is_exact_hessian():
    # b = n with permutation buckets: S_i S_i^T = I, H = A D A^T
    rng = np.random.default_rng(13)
    m, n, N = 96, 512, 2
    A = rng.standard_normal((m, n)).astype(np.float32)
    d = np.exp(rng.uniform(np.log(1e-3), np.log(1e3), size=n)).astype(np.float32)
    h = np.stack([rng.permutation(n) for _ in range(N)]).astype(np.int32)
    s = rng.choice(np.array([-1, 1], np.int8), size=(N, n))
    gb = osk.GramBatch([dev(A)], [dev(d)], b=n, N=N, e=0,
                       hs=[torch.from_numpy(h).cuda()], sigmas=[torch.from_numpy(s).cuda()])
    H = host(gb.run()[0])
    A64, d64 = A.astype(np.float64), d.astype(np.float64)
    assert oracle.rel_frob(H, (A64 * d64) @ A64.T) <= TOL


def test_gram_batch_autotune_reuse_and_graph_replays():
    probs = _problems(SPECS[:2] + SPECS[4:], 14)
    gb = _batch(probs, tile=256)
    eager = [host(h) for h in gb.run()]
    ms = gb.autotune(reps=1)
    assert ms > 0 and gb.config[0] in (MIXED, 128, 256)
    # tile form x grid: three forms, each at one and two times the resident grid
    cands = gb.candidates
    assert len(cands) == 6 and sorted({c[0] for c in cands}) == sorted([MIXED, 128, 256])
    assert all(c[2] > 0 for c in cands)
    best = min(cands, key=lambda c: c[2])
    assert ms == best[2] and gb.config == (best[0], best[1])
    tuned = [host(h) for h in gb.run()]
    for a, b in zip(eager, tuned):
        assert oracle.rel_frob(b, a) <= 1e-6
    from paper_1811_02653_amd.gram import PRODUCT, SKETCH
    again = [host(h) for h in gb.run(stages=SKETCH | PRODUCT)]
    for a, b in zip(tuned, again):
        assert np.array_equal(a, b)
    for h in gb.H:
        h.zero_()
    again = [host(h) for h in gb.run(stages=PRODUCT)]
    for a, b in zip(tuned, again):
        assert np.array_equal(a, b)
    g = gb.graph()
    side = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        for h in gb.H:
            h.fill_(float("nan"))          # eager work between replays
        side = side @ side.T / 512.0
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for a, h in zip(tuned, gb.H):
            assert np.array_equal(a, host(h)), rep
    g.close()
    gr = gb.graph(stages=SKETCH | PRODUCT)
    for h in gb.H:
        h.zero_()
    gr.launch()
    for a, h in zip(tuned, gb.H):
        assert np.array_equal(a, host(h))
    gr.close()
    gb.close()


def test_gram_batch_errors():
    A = torch.zeros(8, 16, device="cuda")
    with pytest.raises(osk.OversketchError):
        osk.GramBatch([A], None, b=4, N=2, e=0, keeps=[np.zeros(2, np.uint8)])
    with pytest.raises(osk.OversketchError):
        osk.GramBatch([A], [torch.zeros(15, device="cuda")], b=4, N=2, e=0)
    gb = osk.GramBatch([A], None, b=4, N=2, e=0)
    with pytest.raises(osk.OversketchError):
        gb.configure(tile=64)
    # a workspace other than the configured one is refused
    other = torch.empty_like(gb.workspace)
    L = osk.lib()
    st = L.os_gram_run(gb._plan, 7, osk._ptr(other), other.numel(),
                       osk._stream())
    assert st == -1
    gb.close()


def test_gram_batch_hessian_workload_sampled():
    # the full batch workload: 64 problems, m_k uniform in [500, 4000],
    # n_k = 20 m_k, b_k = ceil(m_k / 2), N = 6, e = 1 with one block dropped,
    # A_k ~ N(0,1) and d_k log-uniform in [1e-6, 1e6], generated on the
    # device, in the configuration the benchmark times (autotuned tiles);
    # sampled entries of three problems against the oracle, each within
    # 1e-4 * sqrt(H_ii H_jj) (the Cauchy-Schwarz scale of an FP32 sum of
    # K*b products).
    count, seed = 64, 2024
    sizes, As, ds = synthetic.hessian_batch_device(count, seed)
    keeps = [synthetic.random_keep(6, 1, seed + k, drop=1) for k in range(count)]
    bs = [(m + 1) // 2 for m in sizes]
    gb = osk.GramBatch(As, ds, b=bs, N=6, e=1, keeps=keeps, seeds=list(range(count)))
    gb.autotune(reps=1)
    gb.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    order = np.argsort(sizes)
    for k in (int(order[0]), int(order[-1]), int(order[count // 2])):
        m = sizes[k]
        rows = rng.integers(0, m, 48)
        cols = rng.integers(0, m, 48)
        rows[:6] = cols[:6]                     # some diagonal entries
        need = np.unique(np.concatenate([rows, cols]))
        loc = {int(r): t for t, r in enumerate(need)}
        Asub = As[k][torch.from_numpy(need).cuda()].double().cpu().numpy()
        d = ds[k].double().cpu().numpy()
        W = Asub * np.sqrt(d)[None, :]
        pr = np.concatenate([rows, rows, cols])
        pc = np.concatenate([cols, rows, cols])
        ref = oracle.sampled_entries(W, np.ascontiguousarray(W.T),
                                     np.array([loc[int(r)] for r in pr]),
                                     np.array([loc[int(c)] for c in pc]),
                                     bs[k], 6, 1, seed=k, keep=keeps[k])
        t = len(rows)
        ref_ij, ref_ii, ref_jj = ref[:t], ref[t:2 * t], ref[2 * t:]
        Hk = gb.H[k]
        ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
        got = Hk[ri, ci].double().cpu().numpy()
        bound = 1e-4 * np.sqrt(ref_ii * ref_jj)
        assert np.all(np.abs(got - ref_ij) <= bound), (k, m, np.max(np.abs(got - ref_ij) / bound))
        assert torch.equal(Hk[ri, ci], Hk[ci, ri])
    gb.close()
