"""FP64 oracle of the learned Newton initial guess (test infrastructure only: imported by
tests/ and nothing else).

Plain NumPy, one layer at a time, written from the definitions:
  forward   H_0 = X, Z_l = H_{l-1} W_l + b_l, H_l = tanh(Z_l) for hidden layers,
            output Y = Z_L (no activation);
  loss      mean over all n * nout entries of (Y - T)^2;
  gradient  back-propagation: dY = 2 (Y - T) / (n nout); for each layer from the last,
            dW_l = H_{l-1}^T dZ_l, db_l = column sums of dZ_l,
            dH_{l-1} = dZ_l W_l^T, dZ_{l-1} = dH_{l-1} (1 - H_{l-1}^2);
  Adam      Kingma and Ba (2015) with bias correction;
  guess     g = 2 y1 - y2 + gain * sigma * Y, features x = [y1 / s, (y1 - y2) / sigma, phase
            features], target T = (y - (2 y1 - y2)) / sigma, where per component c
            sigma[c] = max(RMS over vertices of (y1 - y2)[:, c], floor[c]); the 21 scales
            are s [7], floor [7], gain [7].
The parameter vector stores W_1, b_1, W_2, b_2, ... with W_l [d_in][d_out] row-major.
Pinned in tests/test_oracle_pins.py by central finite differences, the closed form of a
single linear layer and the closed form of a first Adam step.
"""
from __future__ import annotations

import numpy as np


def layer_dims(nin: int, hidden: int, nlayers: int, nout: int) -> list[tuple[int, int]]:
    return [(nin if l == 0 else hidden, nout if l == nlayers - 1 else hidden) for l in range(nlayers)]


def nparams(dims) -> int:
    return sum(a * b + b for a, b in dims)


def unpack(p, dims):
    out, o = [], 0
    for a, b in dims:
        W = np.asarray(p[o:o + a * b], dtype=np.float64).reshape(a, b)
        o += a * b
        bias = np.asarray(p[o:o + b], dtype=np.float64)
        o += b
        out.append((W, bias))
    return out


def forward(p, dims, X):
    """Activations [H_0 = X, H_1, ..., H_L = Y]."""
    H = [np.asarray(X, dtype=np.float64)]
    layers = unpack(p, dims)
    for l, (W, b) in enumerate(layers):
        Z = H[-1] @ W + b
        H.append(np.tanh(Z) if l + 1 < len(layers) else Z)
    return H


def loss_grad(p, dims, X, T):
    H = forward(p, dims, X)
    Y = H[-1]
    T = np.asarray(T, dtype=np.float64)
    cnt = Y.size
    loss = float(np.sum((Y - T) ** 2) / cnt)
    layers = unpack(p, dims)
    grads = [None] * len(layers)
    dZ = 2.0 * (Y - T) / cnt
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (H[l].T @ dZ, dZ.sum(axis=0))
        if l > 0:
            dH = dZ @ W.T
            dZ = dH * (1.0 - H[l] ** 2)
    g = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss, g


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1 is the step number after this update)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def step_sigma(y1, y2, scales):
    d = np.asarray(y1, dtype=np.float64).reshape(-1, 7) - np.asarray(y2, dtype=np.float64).reshape(-1, 7)
    floor = np.asarray(scales, dtype=np.float64)[7:14]
    return np.maximum(np.sqrt(np.mean(d * d, axis=0)), floor)


def features(y1, y2, scales, tfeat):
    y1 = np.asarray(y1, dtype=np.float64).reshape(-1, 7)
    y2 = np.asarray(y2, dtype=np.float64).reshape(-1, 7)
    s = np.asarray(scales, dtype=np.float64)
    X = np.empty((y1.shape[0], 18))
    X[:, 0:7] = y1 / s[0:7]
    X[:, 7:14] = (y1 - y2) / step_sigma(y1, y2, scales)
    X[:, 14:18] = np.asarray(tfeat, dtype=np.float64)[None, :]
    return X


def target(y, y1, y2, scales):
    ext = 2.0 * np.asarray(y1).reshape(-1, 7) - np.asarray(y2).reshape(-1, 7)
    return (np.asarray(y).reshape(-1, 7) - ext) / step_sigma(y1, y2, scales)


def guess(y1, y2, out, scales):
    s = np.asarray(scales, dtype=np.float64)
    ext = 2.0 * np.asarray(y1).reshape(-1, 7) - np.asarray(y2).reshape(-1, 7)
    if out is None:
        return ext.ravel()
    corr = s[14:21] * step_sigma(y1, y2, scales) * np.asarray(out, dtype=np.float64).reshape(-1, 7)
    return (ext + corr).ravel()
