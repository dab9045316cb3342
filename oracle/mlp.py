"""CPU reference of the surrogate network (test infrastructure only).

Plain numpy in binary64.  Only the test suite may use it; it shares no code
with the HIP implementation.

Network: 7 inputs -> 4 hidden layers of 256 with SiLU -> 4 outputs (an
escape logit and a 3-vector correction of the end direction).  Parameters are
one packed float vector: for each layer, W (in x out, row-major) then b (out).

Loss over a batch of n rays with targets (escaped, d_x, d_y, d_z):
    L = (1/n) sum [ softplus(y0) - escaped * y0
                    + lam * w * sum_c huber(y[c] - d[c]) ]
with huber(e) = e^2 for |e| <= delta and 2 delta |e| - delta^2 beyond
(binary cross-entropy with logits for the class; a squared error of the
direction correction that grows only linearly for outliers, with weight
w = escaped for rows whose target |d| <= dmax and 0 otherwise; delta = inf
gives the plain squared error, dmax = inf keeps every escaped row).

bf16=True rounds, like the GPU kernels, the weights, every layer's input
activations and the activation gradients fed to the backward products to
bfloat16 (round to nearest even); sums stay exact-ish (binary64 here, binary32
on the GPU).

Parity status: pinned by a central-difference gradient check (binary64, no
rounding), closed-form loss values and gradients of an all-zero network, and
Adam's closed-form first step.
"""
from __future__ import annotations

import numpy as np

SIZES = (7, 256, 256, 256, 256, 4)


def num_params(sizes=SIZES) -> int:
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def unpack(params, sizes=SIZES):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = params[o:o + a * b].reshape(a, b)
        o += a * b
        bias = params[o:o + b]
        o += b
        out.append((W, bias))
    assert o == params.size
    return out


def bf16(x):
    """Round binary64 values to bfloat16 (nearest even), returned as binary64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, bf16_mode=False, keep=False):
    """y = MLP(x); with keep=True also returns the per-layer (input, z)."""
    layers = unpack(np.asarray(params, np.float64))
    h = np.asarray(x, np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        if bf16_mode:
            h, W = bf16(h), bf16(W)
        z = h @ W + b
        cache.append((h, z))
        h = silu(z) if li < len(layers) - 1 else z
    return (h, cache) if keep else h


def huber(e, delta):
    if not np.isfinite(delta):
        return e * e
    a = np.abs(e)
    return np.where(a <= delta, e * e, 2.0 * delta * a - delta * delta)


def huber_grad(e, delta):
    if not np.isfinite(delta):
        return 2.0 * e
    return np.where(np.abs(e) <= delta, 2.0 * e, 2.0 * delta * np.sign(e))


def loss_and_grad(params, x, target, lam=100.0, bf16_mode=False, delta=np.inf, dmax=np.inf):
    """Mean loss over the batch and its gradient w.r.t. the packed params.
    Rows whose target correction is longer than dmax take no direction loss."""
    params = np.asarray(params, np.float64)
    layers = unpack(params)
    y, cache = forward(params, x, bf16_mode, keep=True)
    n = y.shape[0]
    esc = target[:, 0]
    d = target[:, 1:4]
    wd = np.where(np.sum(d * d, axis=1) <= dmax * dmax, esc, 0.0)
    sp = np.logaddexp(0.0, y[:, 0])
    e = y[:, 1:4] - d
    L = np.sum(sp - esc * y[:, 0] + lam * wd * np.sum(huber(e, delta), axis=1)) / n
    dy = np.zeros_like(y)
    dy[:, 0] = (sigmoid(y[:, 0]) - esc) / n
    dy[:, 1:4] = lam * wd[:, None] * huber_grad(e, delta) / n
    grads = []
    dz = dy
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h, _z = cache[li]
        if bf16_mode:
            dz = bf16(dz)
            W = bf16(W)
        gW = h.T @ dz
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            dh = dz @ W.T
            dz = dh * silu_grad(cache[li - 1][1])
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def init_params(seed, sizes=SIZES):
    """He-uniform weights (bound sqrt(6/in)), zero biases (reference init)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        bound = np.sqrt(6.0 / a)
        parts.append(rng.uniform(-bound, bound, a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias correction; returns new
    (params, m, v).  t is the 1-based step number."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
