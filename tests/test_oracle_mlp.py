"""Pins of the rank-predictor oracle (FP64): hand-written backpropagation
against central finite differences, the network reducing to an explicit
linear map when every ReLU is active, Adam's first step, and a fit that
learns a smooth target."""
import numpy as np

from oracle import mlp


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.N_IN))
    t = np.log1p((X ** 2).sum(axis=1)) + 0.3 * X[:, 0]
    return X, t


def test_gradient_matches_finite_differences():
    X, t = _data(32, 1)
    p = mlp.init(3)
    p[mlp.N_H * mlp.N_IN:mlp.N_H * mlp.N_IN + mlp.N_H] = 0.05   # b1 > 0: fewer kinks near samples
    L, g = mlp.grad(p, X, t)
    rng = np.random.default_rng(5)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    assert abs(L - mlp.loss(p, X, t)) < 1e-15


def test_all_relus_active_is_a_linear_map():
    rng = np.random.default_rng(2)
    W1 = rng.uniform(0.0, 1.0, (mlp.N_H, mlp.N_IN))
    W2 = rng.uniform(0.0, 1.0, (mlp.N_H, mlp.N_H))
    W3 = rng.standard_normal(mlp.N_H)
    b1 = rng.uniform(0.0, 1.0, mlp.N_H)
    b2 = rng.uniform(0.0, 1.0, mlp.N_H)
    b3 = np.array([0.7])
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = rng.uniform(0.0, 1.0, (10, mlp.N_IN))
    y, _ = mlp.forward(p, X)
    lin = X @ (W3 @ W2 @ W1) + W3 @ W2 @ b1 + W3 @ b2 + b3[0]
    assert np.abs(y - lin).max() < 1e-10 * np.abs(lin).max()
    # then d loss / d b3 = mean(2 (y - t))
    t = np.zeros(10)
    _, g = mlp.grad(p, X, t)
    assert abs(g[-1] - np.mean(2 * y)) < 1e-12 * abs(np.mean(2 * y))


def test_adam_first_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-7)


def test_training_fits_a_smooth_target():
    X, t = _data(2048, 7)
    rng = np.random.default_rng(11)
    order = np.concatenate([rng.permutation(X.shape[0]) for _ in range(30)])
    p, losses = mlp.train(X, t, order, batch=128, lr=3e-3, seed=1)
    assert losses[-20:].mean() < 0.05 * losses[:5].mean()
    assert mlp.loss(p, X, t) < 0.02


def test_seeded_initial_weights_share_the_oracle_layout():
    """The input generator's initial parameters (used by the benchmark) are
    the oracle's He-normal draw in the same packing, rounded to float32."""
    from synth import workloads as W
    for seed in (0, 5):
        a = W.mlp_initial_weights(seed)
        assert a.dtype == np.float32 and a.size == mlp.N_PARAMS
        assert np.array_equal(a, mlp.init(seed).astype(np.float32))
