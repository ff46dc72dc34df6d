"""Seeded input generators: draw order and the torch evaluator of the
Gaussian-source right-hand sides."""
import numpy as np
import torch

from paper_2103_07329_amd import inputs


def test_gaussian_draw_order():
    N, m = 8, 3
    c, s, a = inputs.gaussian_params(N, m, 77)
    rng = np.random.default_rng(77)
    for j in range(m):
        assert np.array_equal(c[j], rng.uniform(0.0, N, size=(8, 3)))
        assert np.array_equal(s[j], rng.uniform(2.0, 8.0, size=8))
        assert np.array_equal(a[j], rng.uniform(-1.0, 1.0, size=8))


def test_gaussian_single_source_value():
    N = 6
    c, s, a = inputs.gaussian_params(N, 1, 5, nsrc=1)
    B = inputs.gaussian_rhs(N, 1, 5, nsrc=1)
    x, y, z = 4, 1, 3
    d2 = (x - c[0, 0, 0]) ** 2 + (y - c[0, 0, 1]) ** 2 + (z - c[0, 0, 2]) ** 2
    assert np.isclose(B[x + N * y + N * N * z, 0], a[0, 0] * np.exp(-d2 / (2 * s[0, 0] ** 2)),
                      rtol=1e-14)


def test_gaussian_torch_matches_numpy():
    N, m = 12, 5
    B = inputs.gaussian_rhs(N, m, 1005)
    params = inputs.gaussian_params(N, m, 1005)
    Bt = inputs.gaussian_rhs_torch(N, params, [3, 0, 4], torch, "cpu").numpy()
    assert np.allclose(Bt, B[:, [3, 0, 4]], rtol=1e-13, atol=1e-15)
