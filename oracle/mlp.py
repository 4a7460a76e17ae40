"""FP64 reference of the learned initial guess's network (not part of the
paper: the learned form predicts the PCG initial guess of eq. (4)'s system).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: per-sample multilayer perceptron with ReLU between layers,
    H_0 = X,  H_l = relu(H_{l-1} W_l^T + b_l) (l < L),  Y = H_{L-1} W_L^T + b_L,
loss = sum over rows m and outputs n < n_valid of  w_m (Y - T)^2_{mn} / (n_rows_valid n_valid),
and Adam (Kingma and Ba, 2015) with bias-corrected moments:
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

``round_bf16`` emulates storage in bfloat16 (round to nearest, ties to even),
the precision in which the GPU keeps weights and activations; with
``bf16_activations`` the forward pass rounds every hidden activation the way
the GPU stores it.

Pinned by: central finite differences of the loss (tests), Adam's first step
(closed form: every parameter moves by lr * sign(g) up to eps), and
bfloat16 rounding against torch's CPU conversion and hand-computed values.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x):
    """Values of float32(x) rounded to bfloat16 (nearest, ties to even), as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = np.where(finite, (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000, u & 0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """uint16 bit patterns of round_bf16(x)."""
    return (np.ascontiguousarray(round_bf16(x).astype(np.float32)).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(h):
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def layer_dims(n_in, width, n_out, n_layers=4):
    dims = [n_in] + [width] * (n_layers - 1) + [n_out]
    return [(dims[i], dims[i + 1]) for i in range(n_layers)]   # (K_l, N_l)


def unpack(theta, n_in, width, n_out):
    """Flat parameter vector -> [(W_l [N][K], b_l [N])] in the library's order."""
    out, off = [], 0
    for k, n in layer_dims(n_in, width, n_out):
        W = np.asarray(theta[off:off + n * k], dtype=np.float64).reshape(n, k)
        off += n * k
        b = np.asarray(theta[off:off + n], dtype=np.float64)
        off += n
        out.append((W, b))
    assert off == len(theta)
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def forward(layers, X, bf16_activations=False):
    """Returns Y and the list of layer inputs (H_0 .. H_{L-1})."""
    H = np.asarray(X, dtype=np.float64)
    inputs = []
    for i, (W, b) in enumerate(layers):
        inputs.append(H)
        Z = H @ W.T + b
        if i < len(layers) - 1:
            H = np.maximum(Z, 0.0)
            if bf16_activations:
                H = round_bf16(H)
        else:
            H = Z
    return H, inputs


def loss_and_grads(layers, X, T, w, n_valid_out, bf16_activations=False):
    """MSE loss of the module docstring and its gradient for every (W_l, b_l)."""
    Y, inputs = forward(layers, X, bf16_activations)
    w = np.asarray(w, dtype=np.float64)
    count = np.count_nonzero(w) * n_valid_out
    D = np.zeros_like(Y)
    D[:, :n_valid_out] = Y[:, :n_valid_out] - T[:, :n_valid_out]
    loss = float(np.sum(w[:, None] * D * D) / count)
    G = 2.0 * w[:, None] * D / count          # dloss / dY
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        Hin = inputs[i]
        grads[i] = (G.T @ Hin, G.sum(axis=0))
        if i > 0:
            G = (G @ W) * (Hin > 0.0)
    return loss, grads


def adam(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t = index of this step, from 1).  Returns theta, m, v."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
