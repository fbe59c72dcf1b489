"""Host checks of the input generators that define the paper's workloads."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")


def test_paper_matrices_and_exact_products():
    m, n, l = 7, 11, 5
    A, B, x, y, z = synthetic.paper_matrices_device(m, n, l, device="cpu")
    i = np.arange(1, m + 1)[:, None]
    k = np.arange(1, n + 1)
    j = np.arange(1, l + 1)[None, :]
    np.testing.assert_array_equal(A.numpy(), (i + k[None, :]).astype(np.float32))
    np.testing.assert_array_equal(B.numpy(), (k[:, None] * j).astype(np.float32))
    Ad, Bd = A.double().numpy(), B.double().numpy()
    # B = A^T
    AB, a2, b2, cross = synthetic.paper_exact_products(x, y)
    np.testing.assert_allclose(AB.numpy(), Ad @ Ad.T, rtol=1e-15)
    assert a2 == pytest.approx(np.sum(Ad ** 2), rel=1e-15) and b2 == a2
    assert cross == pytest.approx(np.sum(np.sum(Ad ** 2, 0) ** 2), rel=1e-14)
    # B(x, y) = x y
    AB, a2, b2, cross = synthetic.paper_exact_products(x, y, z)
    np.testing.assert_allclose(AB.numpy(), Ad @ Bd, rtol=1e-15)
    assert b2 == pytest.approx(np.sum(Bd ** 2), rel=1e-15)
    assert cross == pytest.approx(np.sum(np.sum(Ad ** 2, 0) * np.sum(Bd ** 2, 1)), rel=1e-14)


def test_random_cmask_drops_e_per_block():
    cm = synthetic.random_cmask(3, 4, 26, 4, seed=5)
    assert cm.shape == (3, 4, 30) and cm.dtype == np.uint8
    assert np.all(cm.sum(axis=2) == 26)
    # independent draws per block, reproducible per seed
    assert len({tuple(np.flatnonzero(cm[i, j] == 0)) for i in range(3) for j in range(4)}) > 1
    np.testing.assert_array_equal(cm, synthetic.random_cmask(3, 4, 26, 4, seed=5))
    assert np.all(synthetic.random_cmask(2, 2, 3, 1, seed=1, drop=0) == 1)
