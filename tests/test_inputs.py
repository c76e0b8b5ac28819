"""The seeded input generator: the bilinear field of the gradient workload (rows of the interpolation
weights sum to one, bilinear functions are reproduced exactly, control values are attained at the
control points) and the reproducibility of every draw."""
import numpy as np

from paper_2507_02809_amd import inputs


def test_bilinear_weights_reproduce_bilinear_functions():
    K, N = inputs.FIELD_K, 37
    W = inputs.bilinear_weights(N, K)
    assert W.shape == (N * N, K * K)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-15, rtol=0)
    assert ((W != 0).sum(axis=1) <= 4).all() and (W >= 0).all()
    xi = np.arange(K) / (K - 1)
    x = inputs.grid_points(N, 1.0)
    for a, b, c, d in [(1.0, 0.0, 0.0, 0.0), (0.3, -2.0, 5.0, 0.0), (0.0, 1.0, 1.0, 7.0)]:
        G = a + b * xi[:, None] + c * xi[None, :] + d * np.outer(xi, xi)
        ref = a + b * x[:, None] + c * x[None, :] + d * np.outer(x, x)
        np.testing.assert_allclose(W @ G.reshape(-1), ref.reshape(-1), rtol=0, atol=1e-13)


def test_bilinear_weights_hit_control_values_on_the_control_grid():
    # N + 1 = 2 (K - 1): every other grid point is a control point
    K = 5
    N = 2 * (K - 1) - 1
    W = inputs.bilinear_weights(N, K)
    G = np.random.default_rng(0).random((K, K))
    f = (W @ G.reshape(-1)).reshape(N, N)
    np.testing.assert_allclose(f[1::2, 1::2], G[1:-1, 1:-1], rtol=0, atol=1e-15)


def test_inputs_are_reproducible():
    a, b = inputs.c5(3), inputs.c5(3)
    for k in ("gamma1", "gamma2", "q", "rho", "f_true", "noise"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert not np.array_equal(inputs.c5(3).gamma2, inputs.c5(4).gamma2)
    g = inputs.c5(0).gamma2
    assert np.array_equal(g[0], g[-1]) and 0.8 <= g.min() and g.max() <= 1.2
