"""Plain FP64 reference of the cost-model network (test infrastructure only).

12 -> 64 -> 64 -> 1 with ReLU; loss = mean squared error.  Written directly
from the definition of a fully connected network and back-propagation, with
numpy matrix products as the only library steps.  Weights are used as given;
callers that compare against the GPU round them to BF16 first with
``bf16_round`` (round to nearest, ties to even), exactly as the GPU does.
"""
from __future__ import annotations

import numpy as np

F, H = 12, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + H * F
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
N_PARAMS = OFF_B3 + 1


def bf16_round(a) -> np.ndarray:
    """Round float32 values to the nearest BF16 value (ties to even)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    return (w[OFF_W1:OFF_B1].reshape(H, F), w[OFF_B1:OFF_W2], w[OFF_W2:OFF_B2].reshape(H, H),
            w[OFF_B2:OFF_W3], w[OFF_W3:OFF_B3], w[OFF_B3])


def forward(w, X):
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    return h2 @ w3 + b3


def loss(w, X, Y):
    return float(np.mean((forward(w, X) - np.asarray(Y, dtype=np.float64)) ** 2))


def grad(w, X, Y):
    """d/dw of mean_s (y_s - t_s)^2, flat FP64 [N_PARAMS]."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n = X.shape[0]
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w3 + b3
    dy = 2.0 * (y - Y) / n                 # dL/dy_s
    g = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = h2.T @ dy
    g[OFF_B3] = dy.sum()
    da2 = np.outer(dy, w3) * (a2 > 0)      # dL/da2
    g[OFF_W2:OFF_B2] = (da2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0)            # dL/da1
    g[OFF_W1:OFF_B1] = (da1.T @ X).ravel()
    g[OFF_B1:OFF_W2] = da1.sum(axis=0)
    return g


def forward_bf16_act(w, X):
    """Forward pass with the inputs and both hidden activations rounded to
    BF16 after the ReLU, as the matrix-core inference path computes them."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X = bf16_round(np.asarray(X, dtype=np.float32)).astype(np.float64)
    h1 = bf16_round(np.maximum(X @ W1.T + b1, 0.0).astype(np.float32)).astype(np.float64)
    h2 = bf16_round(np.maximum(h1 @ W2.T + b2, 0.0).astype(np.float32)).astype(np.float64)
    return h2 @ w3 + b3
