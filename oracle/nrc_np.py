"""FP64 numpy oracle of the radiance-cache network (test infrastructure only).

Network (the reading of neural radiance caching, named by the paper as
future work in Sec. 6.1): 64 encoded features -> 5 hidden layers of 64 with
ReLU -> 3 linear outputs, no biases.  Parameters W0..W4 (64 x 64) and
W5 (3 x 64), row-major [out][in], concatenated: 20,672 values.

* forward: z_l = W_l a_l, a_{l+1} = max(z_l, 0) for l = 0..4; y = W5 a_5.
* loss: relative L2, mean over samples and channels of
  (y - t)^2 / (sg(y)^2 + 0.01), sg = no gradient through the denominator.
* backward: g_5 = dL/dy; dW_l = sum_n g_l a_l^T; g_{l-1} = (W_l^T g_l) * [z_{l-1} > 0].
* Adam (Kingma & Ba) with bias correction: lr 1e-3, beta1 0.9, beta2 0.99, eps 1e-8.
* Inference weights: bias-corrected exponential moving average of the
  weights over the Adam steps (decay in [0, 1); 0 = the weights).
* He-uniform initialisation: weight k of layer l is (2u - 1) sqrt(6 / 64)
  with u the Philox uniform at (pixel k, sample l, bounce 0x4E5243, dim 0).

With bf16=True the tensor operands are rounded to bfloat16 as the GPU's
matrix-core inputs are (weights, encoded input, hidden activations, and
each layer's output gradient); sums stay FP64.
"""
from __future__ import annotations

import numpy as np

WIDTH = 64
N_HIDDEN = 5
N_OUT = 3
N_PARAMS = N_HIDDEN * WIDTH * WIDTH + N_OUT * WIDTH  # 20672
INIT_STREAM = 0x4E5243


def bf16(a):
    """Round to bfloat16 (nearest even) and back to float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = np.where(finite, r, u).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == N_PARAMS
    mats = [w[l * 4096:(l + 1) * 4096].reshape(64, 64) for l in range(N_HIDDEN)]
    mats.append(w[N_HIDDEN * 4096:].reshape(N_OUT, 64))
    return mats


def pack(mats):
    return np.concatenate([m.reshape(-1) for m in mats])


def encode(X):
    """[N, 12] cache inputs -> [N, 64] features."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    F = np.zeros((N, 64))
    for a in range(3):
        for k in range(6):
            w = np.ldexp(np.pi, k) * X[:, a]
            F[:, 12 * a + 2 * k] = np.sin(w)
            F[:, 12 * a + 2 * k + 1] = np.cos(w)

    def blob(s, i, periodic=False):
        d = s - (i + 0.5) / 4.0
        if periodic:  # the azimuths wrap: 0 and 1 are the same direction
            d = d - np.floor(d + 0.5)
        z = d * 4.0
        return np.exp(-0.5 * z * z)

    for c in range(4):
        for i in range(4):
            F[:, 36 + 4 * c + i] = blob(X[:, 3 + c], i, periodic=(c % 2 == 1))
    rr = 1.0 - np.exp(-X[:, 7])
    for i in range(4):
        F[:, 52 + i] = blob(rr, i)
    F[:, 56:60] = X[:, 8:12]
    F[:, 60] = 1.0
    return F


def forward(w, X, use_bf16=False):
    """Returns y [N, 3] and the cache (a_0..a_5 layer inputs, z_0..z_4)."""
    W = unpack(w)
    r = bf16 if use_bf16 else (lambda v: v)
    a = r(encode(X))
    acts, zs = [a], []
    for l in range(N_HIDDEN):
        z = a @ r(W[l]).T
        zs.append(z)
        a = r(np.maximum(z, 0.0))
        acts.append(a)
    y = a @ r(W[N_HIDDEN]).T
    return y, (acts, zs)


def loss_and_grad(y, t):
    """Relative L2 loss and dL/dy (denominator treated as a constant)."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    d = y * y + 0.01
    n = y.size
    loss = float(np.sum((y - t) ** 2 / d) / n)
    return loss, 2.0 * (y - t) / d / n


def backward(w, cache, dy, use_bf16=False):
    """Gradient of the loss w.r.t. all 20,672 weights, given dL/dy."""
    W = unpack(w)
    acts, zs = cache
    r = bf16 if use_bf16 else (lambda v: v)
    grads = [None] * (N_HIDDEN + 1)
    g = r(dy)
    grads[N_HIDDEN] = g.T @ acts[N_HIDDEN]
    for l in range(N_HIDDEN - 1, -1, -1):
        g = r((g @ r(W[l + 1])) * (zs[l] > 0.0))
        grads[l] = g.T @ acts[l]
    return pack(grads)


def loss_fn(w, X, t, use_bf16=False):
    y, _ = forward(w, X, use_bf16)
    return loss_and_grad(y, t)[0]


def gradient(w, X, t, use_bf16=False):
    y, cache = forward(w, X, use_bf16)
    loss, dy = loss_and_grad(y, t)
    return loss, backward(w, cache, dy, use_bf16)


def adam(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.99, eps=1e-8):
    """One Adam update; step counts from 1.  Returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def ema_update(e, w, alpha):
    """Moving average of the weights after an Adam step: e = alpha e + (1 - alpha) w
    (e starts at zero).  The cited cache method renders with such an average of
    the weights rather than the latest ones (Sec. 6.1 names the method)."""
    return alpha * np.asarray(e, dtype=np.float64) + (1.0 - alpha) * np.asarray(w, dtype=np.float64)


def ema_weights(e, t, alpha, w):
    """Inference weights after t Adam steps: the bias-corrected average
    e / (1 - alpha^t); the weights w themselves when alpha is 0 or t is 0."""
    if alpha == 0.0 or t == 0:
        return np.asarray(w, dtype=np.float64)
    return np.asarray(e, dtype=np.float64) / (1.0 - alpha ** t)


def init_weights(seed, uniform):
    """He-uniform weights; `uniform(seed, pixel, sample, bounce, dim)` is the Philox uniform."""
    w = np.zeros(N_PARAMS)
    scale = np.sqrt(6.0 / 64.0)
    off = 0
    for l in range(N_HIDDEN + 1):
        n = 4096 if l < N_HIDDEN else N_OUT * 64
        for k in range(n):
            w[off + k] = (2.0 * uniform(seed, k, l, INIT_STREAM, 0) - 1.0) * scale
        off += n
    return w
