"""Pins of the FP64 reference network of the learned initial guess:
central finite differences of the loss, Adam's first step in closed form, and
bfloat16 rounding against torch's CPU conversion and hand-computed values."""
import numpy as np
import pytest

from oracle import mlp


def tiny(seed=0, n_in=6, width=8, n_out=4, rows=11):
    rng = np.random.default_rng(seed)
    layers = []
    for k, n in mlp.layer_dims(n_in, width, n_out):
        layers.append((rng.standard_normal((n, k)) / np.sqrt(k), 0.1 * rng.standard_normal(n)))
    X = rng.standard_normal((rows, n_in))
    T = rng.standard_normal((rows, n_out))
    w = np.ones(rows)
    w[[2, 7]] = 0.0
    return layers, X, T, w


def test_gradients_match_central_differences():
    layers, X, T, w = tiny()
    n_valid = 3
    _, grads = mlp.loss_and_grads(layers, X, T, w, n_valid)
    theta = mlp.pack(layers)
    g_an = mlp.pack(grads)
    h = 1e-6
    g_fd = np.zeros_like(theta)
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = mlp.loss_and_grads(mlp.unpack(tp, 6, 8, 4), X, T, w, n_valid)
        lm, _ = mlp.loss_and_grads(mlp.unpack(tm, 6, 8, 4), X, T, w, n_valid)
        g_fd[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(g_an - g_fd) <= 1e-6 * np.linalg.norm(g_fd)
    # outputs past n_valid and rows of weight 0 carry no gradient
    W4g, b4g = grads[-1]
    assert not np.any(W4g[n_valid:]) and not np.any(b4g[n_valid:])
    X2 = X.copy()
    X2[[2, 7]] += 5.0
    _, grads2 = mlp.loss_and_grads(layers, X2, T, w, n_valid)
    assert np.allclose(mlp.pack(grads2), g_an)


def test_adam_first_step_moves_by_lr_sign():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    new, m, v = mlp.adam(theta, g, z, z, 1, lr=1e-3, eps=0.0)
    assert np.allclose(new - theta, -1e-3 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_bf16(x), ref)
    # ties go to the even neighbour: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert mlp.round_bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert mlp.round_bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6
    assert mlp.bf16_bits(np.float32(1.0)) == 0x3F80
    assert np.array_equal(mlp.from_bf16_bits(mlp.bf16_bits(x)), mlp.round_bf16(x))
