"""Run-to-run determinism of the whole path: the same inputs and seed give
bitwise-identical C on repeated calls, for the global-mask product in every
operand precision, with and without kept_only, and for per-C-block masks.

Every bucket of every line is summed by one lane in a fixed order and every
C tile by one workgroup in a fixed K order (no atomics, no split-K), so the
result does not depend on scheduling; these tests hold the library to it.
Between the calls other work runs on the GPU and a fresh workspace is used.
"""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1811_02653_amd as osk  # noqa: E402

# several sketch windows (n > 8192), two sketch passes for the wide case,
# ragged edges everywhere
CASES = [(300, 20000, 200, 256, 4, 2), (130, 9001, 517, 100, 3, 1), (64, 3000, 40, 2048, 8, 2)]


def _disturb():
    # unrelated work between the calls (other kernels, allocator churn)
    x = torch.randn(1 << 20, device="cuda")
    (x * 2).sum().item()


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp8", "fp8x3"])
@pytest.mark.parametrize("kept_only", [False, True])
@pytest.mark.parametrize("m,n,l,b,N,e", CASES)
def test_matmul_bitwise_repeatable(m, n, l, b, N, e, kept_only, precision):
    seed = m + n + l
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    keep = synthetic.random_keep(N, e, seed)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    outs = []
    for _ in range(3):
        outs.append(osk.matmul(Ad, Bd, b, N, e, seed=seed, keep=keep, kept_only=kept_only,
                               precision=precision))
        _disturb()
    torch.cuda.synchronize()
    assert torch.isfinite(outs[0]).all()
    for C in outs[1:]:
        assert torch.equal(C, outs[0])


@pytest.mark.parametrize("b_layout", ["row", "col"])
def test_matmul_ex_bf16_operands_bitwise_repeatable(b_layout):
    m, n, l, b, N, e, seed = 200, 12000, 96, 512, 4, 0, 9
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    Ad = torch.from_numpy(A).cuda().bfloat16()
    Bd = torch.from_numpy(B).cuda().bfloat16()
    if b_layout == "col":
        Bd = Bd.t().contiguous().t()
    outs = []
    for _ in range(2):
        outs.append(osk.matmul_ex(Ad, Bd, b, N, e, seed=seed, kept_only=True,
                                  precision="bf16"))
        _disturb()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("m,n,l,b,N,e", [(300, 20000, 200, 128, 4, 2), (513, 5000, 260, 256, 3, 1)])
def test_matmul_cmask_bitwise_repeatable(m, n, l, b, N, e):
    seed = 17 + m
    A, B = synthetic.gaussian_pair(m, n, l, seed)
    cmask = synthetic.random_cmask(-(-m // b), -(-l // b), N, e, seed)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    outs = []
    for _ in range(3):
        outs.append(osk.matmul_cmask(Ad, Bd, b, N, e, cmask, seed=seed))
        _disturb()
    torch.cuda.synchronize()
    for C in outs[1:]:
        assert torch.equal(C, outs[0])


def test_distinct_seeds_give_distinct_products():
    # (the repeatability above is not vacuous: the result does depend on S)
    m, n, l, b, N, e = 64, 4096, 64, 128, 2, 0
    A, B = synthetic.gaussian_pair(m, n, l, 1)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C1 = osk.matmul(Ad, Bd, b, N, e, seed=1)
    C2 = osk.matmul(Ad, Bd, b, N, e, seed=2)
    torch.cuda.synchronize()
    assert not torch.equal(C1, C2)
