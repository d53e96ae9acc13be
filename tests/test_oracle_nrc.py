"""Pins of the radiance-cache oracle (CPU only).

The encoding and network are written twice (C in oracle/nrc.c for the path
tracer, numpy in oracle/nrc_np.py for training) and checked against each
other; both are pinned by closed forms: trigonometric identities of the
frequency features, one-blob values at bin centres, a network of
permutation matrices whose output follows from index bookkeeping, central
finite differences of the loss, Adam's first step, and the white furnace
seen through a cache that returns 1.
"""
import math

import numpy as np
import pytest

from oracle import nrc_np as N
from paper_2407_19977_amd import scenes


def _inputs(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    X = np.zeros((n, 12))
    X[:, 0:3] = r.uniform(0, 1, (n, 3))
    X[:, 3:7] = r.uniform(0, 1, (n, 4))
    X[:, 7] = r.uniform(0, 1, n)
    X[:, 8:12] = r.uniform(0, 1, (n, 4))
    return X


def test_encoding_c_equals_numpy_and_identities(O):
    X = _inputs(200, 1)
    F = N.encode(X)
    for i in range(200):
        assert np.allclose(O.nrc_encode(X[i]), F[i], atol=1e-15, rtol=0)
    for a in range(3):
        for k in range(6):
            s, c = F[:, 12 * a + 2 * k], F[:, 12 * a + 2 * k + 1]
            assert np.allclose(s * s + c * c, 1.0, atol=1e-14)
            if k < 5:  # double angle: sin(2w) = 2 sin(w) cos(w)
                assert np.allclose(F[:, 12 * a + 2 * k + 2], 2 * s * c, atol=1e-12)
    # one-blob: value 1 at the centre of its bin, exp(-1/2) at the neighbouring bins' centres
    x = np.zeros((4, 12))
    for i in range(4):
        x[i, 3] = (i + 0.5) / 4
    f = N.encode(x)[:, 36:40]
    assert np.allclose(np.diag(f), 1.0, atol=1e-15)
    for i in range(3):
        assert abs(f[i, i + 1] - math.exp(-0.5)) < 1e-15 and abs(f[i + 1, i] - math.exp(-0.5)) < 1e-15
    assert np.all(F[:, 60] == 1) and np.all(F[:, 61:64] == 0)
    assert np.array_equal(F[:, 56:60], X[:, 8:12])
    assert np.all(np.abs(F) <= 1.0 + 1e-15)


def _perm_weights(seed):
    r = np.random.Generator(np.random.PCG64(seed))
    sig = [r.permutation(64) for _ in range(5)]
    mats = []
    for s in sig:
        P = np.zeros((64, 64))
        P[np.arange(64), s] = 1.0     # row i picks input s[i]
        mats.append(P)
    pick = r.choice(64, 3, replace=False)
    W5 = np.zeros((3, 64))
    W5[np.arange(3), pick] = 1.0
    mats.append(W5)
    return N.pack(mats), sig, pick


def test_forward_permutation_network_closed_form(O):
    w, sig, pick = _perm_weights(4)
    X = _inputs(64, 2)
    F = N.encode(X)
    # a_5[i] = relu(a_0[s0[s1[s2[s3[s4[i]]]]]]) by index bookkeeping
    idx = np.arange(64)
    for s in reversed(sig):
        idx = s[idx]
    expect = np.maximum(F[:, idx[pick]], 0.0)
    y, _ = N.forward(w, X)
    assert np.allclose(y, expect, atol=1e-15)
    for i in range(0, 64, 7):
        assert np.allclose(O.nrc_forward(w, X[i]), expect[i], atol=1e-15)


def test_forward_c_equals_numpy_random_weights(O):
    w = N.init_weights(7, O.uniform)
    X = _inputs(50, 3)
    for bf in (False, True):
        y, _ = N.forward(w, X, use_bf16=bf)
        for i in range(50):
            assert np.allclose(O.nrc_forward(w, X[i], bf16=bf), y[i], rtol=1e-12, atol=1e-14)


def test_gradient_matches_central_differences(O):
    r = np.random.Generator(np.random.PCG64(5))
    w = N.init_weights(11, O.uniform)
    X = _inputs(12, 6)
    t = r.uniform(0, 2, (12, 3))
    loss, g = N.gradient(w, X, t)
    assert loss > 0
    # the denominator sg(y)^2 + 0.01 carries no gradient: hold it at the base point
    y0, _ = N.forward(w, X)
    d0 = y0 * y0 + 0.01

    def frozen(wv):
        y, _ = N.forward(wv, X)
        return float(np.sum((y - t) ** 2 / d0) / y.size)

    assert abs(frozen(w) - loss) < 1e-15
    h = 1e-6
    coords = np.concatenate([r.choice(4096, 8, replace=False) + 4096 * l for l in range(5)] +
                            [20480 + r.choice(192, 8, replace=False)])
    for k in coords:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (frozen(wp) - frozen(wm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_loss_zero_at_target_and_adam_first_step(O):
    w = N.init_weights(3, O.uniform)
    X = _inputs(8, 9)
    y, _ = N.forward(w, X)
    loss, dy = N.loss_and_grad(y, y)
    assert loss == 0.0 and np.all(dy == 0)
    r = np.random.Generator(np.random.PCG64(1))
    g = r.normal(size=N.N_PARAMS)
    w1, m1, v1 = N.adam(w, np.zeros_like(w), np.zeros_like(w), g, 1)
    # bias-corrected first step: -lr g / (|g| + eps)
    assert np.allclose(w1 - w, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    w1b, _, _ = N.adam(w, np.zeros_like(w), np.zeros_like(w), 37.0 * g, 1)
    big = np.abs(g) > 1e-2  # invariant to the gradient's scale (up to eps)
    assert np.allclose((w1b - w)[big], (w1 - w)[big], rtol=1e-5, atol=0)


def test_init_is_he_uniform(O):
    w = N.init_weights(0, O.uniform)
    b = math.sqrt(6 / 64)
    assert np.all(np.abs(w) <= b) and abs(w.mean()) < 0.01
    assert abs(w.var() - b * b / 3) < 0.02 * b * b


def _constant_cache(value):
    """Hidden layers pass the constant feature (index 60) through, the output is value * it."""
    mats = [np.zeros((64, 64)) for _ in range(5)]
    for M in mats:
        M[60, 60] = 1.0
    W5 = np.zeros((3, 64))
    W5[:, 60] = value
    return N.pack(mats + [W5])


def test_furnace_through_a_unit_cache_is_exact(O):
    """Convex white object under a uniform sky of 1 with a cache returning 1 at the
    first hit: every pixel is exactly 1 (the query adds beta * 1 and ends the path)."""
    sc = scenes.furnace("sphere", width=16, height=16)
    os_ = O.OracleScene(sc)
    r = os_.render(4, 5, per_sample=True, nrc_weights=_constant_cache(1.0), nrc_bounce=0)
    assert np.allclose(r["per_sample"], 1.0, atol=1e-12)
    # a cache returning 0.5 scales only the pixels that see the object
    r2 = os_.render(4, 5, per_sample=True, nrc_weights=_constant_cache(0.5), nrc_bounce=0)
    v = r2["per_sample"].reshape(-1, 3)
    assert np.all(np.isclose(v, 1.0, atol=1e-12) | np.isclose(v, 0.5, atol=1e-12))
    assert np.isclose(v, 0.5).mean() > 0.05


def test_training_targets_are_outgoing_radiance(O):
    """White furnace: the outgoing radiance of the object (no emission) is 1 in every
    direction, so the targets recorded at its vertices average to 1."""
    sc = scenes.furnace("sphere", width=16, height=16)
    os_ = O.OracleScene(sc)
    tg = []
    for s in range(64):
        for y in range(16):
            for x in range(16):
                X, T = os_.training_records(x, y, s, 6)
                if len(T):
                    assert np.all(X[:, 0:3] >= -1e-12) and np.all(X[:, 0:3] <= 1 + 1e-12)
                    tg.append(T)
    tg = np.concatenate(tg)
    assert len(tg) > 3000
    m, se = tg.mean(0), tg.std(0) / math.sqrt(len(tg))
    assert np.all(np.abs(m - 1.0) < 4 * se)
