"""The batched workload's input recipe: shape distribution and exact spectra."""
import numpy as np

from synthetic import batch_shapes, batch_spectral


def test_batch_shapes_distribution():
    sh = np.array(batch_shapes(4096, seed=0))
    m, n = sh[:, 0], sh[:, 1]
    assert n.min() >= 64 and n.max() <= 512 and np.all(m >= n) and np.all(m <= 2 * n)
    # roughly uniform: every eighth of [64, 512] holds 1/8 of the batch (+-25%)
    hist, _ = np.histogram(n, bins=8, range=(64, 513))
    assert np.all(np.abs(hist - 512) < 128)
    assert batch_shapes(16, seed=0) == batch_shapes(16, seed=0)


def test_batch_spectral_singular_values():
    shapes = batch_shapes(12, seed=3, nmin=8, nmax=60)
    for (m, n), A in zip(shapes, batch_spectral(shapes, seed=3, decades=8.0)):
        assert A.shape == (m, n) and A.flags.f_contiguous
        s = np.linalg.svd(A, compute_uv=False)
        want = 10.0 ** (-8.0 * np.arange(n) / (n - 1))
        np.testing.assert_allclose(s, want, rtol=0, atol=1e-14)
