"""FP64 reference of the learned warm start -- TEST INFRASTRUCTURE ONLY.

The warm start predicts initial weights W_0 for Algorithm 2 (which starts
from W_0 = 0 in the paper) from per-seed features.  This module is the
plain NumPy reading of what the GPU kernels compute, used to check them:

* features (2D): for seed i, its own (x_i, the upper triangle of A_i, N v_i),
  the mean over its 16 nearest seeds (Euclidean, ties to the lower index)
  of (sqrt(N) (x_j - x_i), the upper triangle of A_j, N v_j,
  N |x_j - x_i|^2_{A_i}, N |x_j - x_i|^2_{A_j}), the distance of x_i to
  the box boundary along each axis times sqrt(N / |Omega|), the volume
  deficit d_i = N (v_i - |C_i|) of the cells at W = 0 (N times the gradient
  of eq. (2.8) at zero weights, an input here), and the 1-, 2- and 3-fold
  repeated means of d over the 16 nearest seeds; 20 numbers;
* the network 20 -> 128 -> 128 -> 128 -> 1 with ReLU between layers; the
  parameters are one flat vector (per layer W [in][out] row-major, then b);
* the loss: mean squared error against t_i = N (w*_i - mean w*) of solver
  weights w* (weights scale like a squared cell radius, ~ 1/N in 2D);
* Adam (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected);
* the prediction: w_i = (y_i - mean y) / N.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(20, 128), (128, 128), (128, 128), (128, 1)]
N_FEAT = 20
K_NEIGH = 16
POOL_HOPS = 3


def n_params() -> int:
    return sum(i * o + o for i, o in LAYERS)


def unpack(params):
    out, k = [], 0
    for i, o in LAYERS:
        W = params[k:k + i * o].reshape(i, o)
        k += i * o
        b = params[k:k + o]
        k += o
        out.append((W, b))
    return out


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (the random draws are an input of the
    GPU side: it receives this vector)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in LAYERS:
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, i * o))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def features(x, A, v, lo=(0.0, 0.0), hi=(1.0, 1.0), d=None) -> np.ndarray:
    """Per-seed features; d is the deficit N (v - |C|) at W = 0 (zeros if
    not given)."""
    x = np.asarray(x, np.float64)
    A = np.asarray(A, np.float64)
    v = np.asarray(v, np.float64)
    n = len(x)
    F = np.zeros((n, N_FEAT))
    F[:, 0:2] = x
    F[:, 2] = A[:, 0, 0]
    F[:, 3] = A[:, 0, 1]
    F[:, 4] = A[:, 1, 1]
    F[:, 5] = n * v
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    sc = np.sqrt(n / np.prod(hi - lo))
    F[:, 14:16] = sc * np.minimum(x - lo, hi - x)
    d = np.zeros(n) if d is None else np.asarray(d, np.float64)
    F[:, 16] = d
    k = min(K_NEIGH, n - 1)
    if k <= 0:
        return F
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    nb = np.argsort(d2, axis=1, kind="stable")[:, :k]       # ties -> lower index
    dx = x[nb] - x[:, None, :]                               # (n, k, 2)
    F[:, 6:8] = np.sqrt(n) * dx.mean(axis=1)
    F[:, 8] = A[nb, 0, 0].mean(axis=1)
    F[:, 9] = A[nb, 0, 1].mean(axis=1)
    F[:, 10] = A[nb, 1, 1].mean(axis=1)
    F[:, 11] = (n * v[nb]).mean(axis=1)
    F[:, 12] = n * np.einsum("nka,nab,nkb->nk", dx, A, dx).mean(axis=1)
    F[:, 13] = n * np.einsum("nka,nkab,nkb->nk", dx, A[nb], dx).mean(axis=1)
    p = d
    for h in range(POOL_HOPS):
        p = p[nb].mean(axis=1)
        F[:, 17 + h] = p
    return F


def deficit(n, grad0) -> np.ndarray:
    """d = N (v - |C|) from the gradient (2.8) of a pass at W = 0."""
    return n * np.asarray(grad0, np.float64)


def forward(params, X):
    """Returns the output y (S,) and the activations of every layer."""
    layers = unpack(np.asarray(params, np.float64))
    h = np.asarray(X, np.float64)
    acts = [h]
    for li, (W, b) in enumerate(layers):
        z = h @ W + b
        h = np.maximum(z, 0.0) if li < len(layers) - 1 else z
        acts.append(h)
    return h[:, 0], acts


def to_bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64:
    the 8 leading bits of the FP32 significand survive."""
    x32 = np.asarray(x, np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params, X):
    """BF16 inference by definition: every layer's weights and inputs are
    rounded to BF16, products and sums are exact (FP64 here), the bias and
    ReLU follow.  Returns y and, per sample, the absolute sum
    sum_o |h_o w_o| + |b| of the output layer (the scale of its rounding)."""
    layers = unpack(np.asarray(params, np.float64))
    h = np.asarray(X, np.float64)
    scale = None
    for li, (W, b) in enumerate(layers):
        a, Wb = to_bf16(h), to_bf16(W)
        z = a @ Wb + b
        if li < len(layers) - 1:
            h = np.maximum(z, 0.0)
        else:
            scale = (np.abs(a) @ np.abs(Wb) + np.abs(b))[:, 0]
            h = z
    return h[:, 0], scale


def loss_and_grad(params, X, t):
    """MSE loss mean((y - t)^2) and its gradient with respect to the flat
    parameter vector (back-propagation written out layer by layer)."""
    params = np.asarray(params, np.float64)
    layers = unpack(params)
    y, acts = forward(params, X)
    S = len(y)
    r = y - np.asarray(t, np.float64)
    loss = float(np.mean(r * r))
    dh = (2.0 / S) * r[:, None]
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        h_in = acts[li]
        gW = h_in.T @ dh
        gb = dh.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            dh = (dh @ W.T) * (acts[li] > 0.0)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def targets(w, n) -> np.ndarray:
    w = np.asarray(w, np.float64)
    return n * (w - w.mean())


def prediction_to_weights(y, n) -> np.ndarray:
    y = np.asarray(y, np.float64)
    return (y - y.mean()) / n
