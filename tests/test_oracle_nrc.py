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
    # the azimuth bins (inputs 4 and 6) are periodic: s = 0 and s = 1 encode alike, bin 3 at s = 0
    # sees the distance 1/8 across the seam, and bin 0 at s = 1 - 1/8 the distance 1/4
    x = np.zeros((3, 12))
    x[:, 4] = x[:, 6] = [0.0, 1.0, 0.875]
    f = N.encode(x)
    for base in (40, 48):
        assert np.allclose(f[0, base:base + 4], f[1, base:base + 4], atol=1e-15)
        assert abs(f[0, base + 3] - math.exp(-0.5 * 0.25)) < 1e-15 and abs(f[0, base] - math.exp(-0.5 * 0.25)) < 1e-15
        assert abs(f[2, base] - math.exp(-0.5)) < 1e-15 and abs(f[2, base + 3] - 1.0) < 1e-15
        for c in range(3):
            assert np.allclose(O.nrc_encode(x[c])[base:base + 4], f[c, base:base + 4], atol=1e-15)
    # the polar angles and the roughness are not periodic
    assert abs(f[0, 36] - math.exp(-0.5 * 0.25)) < 1e-15 and abs(f[0, 39] - math.exp(-0.5 * 3.5 ** 2)) < 1e-15
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


# ------------------------------------------------- self-training, factorisation --

def _box_paths(os_, n_paths, fn):
    for k in range(n_paths):
        px, py, smp = (7 * k) % 32, (11 * k) % 32, k // 7
        yield k, fn(px, py, smp)


def test_self_training_with_a_zero_cache_is_the_truncated_path(O):
    """A training path that ends in a cache answering 0 at vertex T carries the
    records and targets of the same path traced plain to max_depth T (its
    vertices before T, the emission found at T, nothing after)."""
    sc = scenes.cornell(width=32, height=32)
    os_ = O.OracleScene(sc)
    zero = np.zeros(N.N_PARAMS)
    seen = 0
    for T in (1, 2, 3):
        for k, (a, b) in _box_paths(os_, 300, lambda px, py, smp: (
                os_.training_records(px, py, smp, 6, nrc_weights=zero, train_end=T),
                os_.training_records(px, py, smp, T))):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            seen += len(a[0])
    assert seen > 500


def test_self_training_adds_the_cache_times_the_albedo_product(O):
    """Lambertian box, roulette off: cosine sampling gives each bounce the
    weight rho(x_j) exactly, so a cache answering c at vertex T raises the
    target of vertex k by c * prod_{j=k}^{T-1} rho(x_j), with rho read from the
    records' diffuse-albedo inputs; a path that leaves the box before T is
    unchanged."""
    sc = scenes.cornell(width=32, height=32)
    os_ = O.OracleScene(sc)
    c = 0.7
    w = _constant_cache(c)
    T = 3
    raised = 0
    for k, (a, b) in _box_paths(os_, 400, lambda px, py, smp: (
            os_.training_records(px, py, smp, 6, nrc_weights=w, train_end=T, rr=False),
            os_.training_records(px, py, smp, T, rr=False))):
        (Xs, Ts), (Xp, Tp) = a, b
        assert np.array_equal(Xs, Xp)
        d = Ts - Tp
        if not np.any(d):
            continue
        assert len(Xs) == T  # the path reached T: every earlier vertex scattered and recorded
        for i in range(T):
            prod = np.prod(Xs[i:T, 8:11], axis=0)
            assert np.allclose(d[i], c * prod, rtol=1e-12, atol=0), (k, i, d[i], c * prod)
        raised += 1
    assert raised > 50


def test_factorised_targets_divide_by_albedo_plus_normal_reflectance(O):
    """The box's Lambert walls have specular_weight 0, so their modulated IOR is
    1 and their specular input F(1, 1) is 0: the reflectance factor is rho per
    channel, and factorised targets are the plain ones divided by it.  A wall
    with specular_weight 1 (IOR 1.5) adds ((1.5 - 1) / (1.5 + 1))^2 = 0.04."""
    sc = scenes.cornell(width=32, height=32)
    os_ = O.OracleScene(sc)
    n = 0
    for k, (a, b) in _box_paths(os_, 200, lambda px, py, smp: (
            os_.training_records(px, py, smp, 5, factorize=True), os_.training_records(px, py, smp, 5))):
        (Xf, Tf), (Xp, Tp) = a, b
        keep = np.all(Xp[:, 8:11] + Xp[:, 11:12] != 0.0, axis=1)  # a zero factor drops the record (the light)
        Xp, Tp = Xp[keep], Tp[keep]
        assert np.array_equal(Xf, Xp)
        assert np.all(Xf[:, 11] == 0.0)
        assert np.allclose(Tf * Xf[:, 8:11], Tp, rtol=1e-12, atol=1e-15)
        n += len(Tf)
    assert n > 300
    # specular_weight 1: the cache input is the normal-incidence reflectance 0.04 of IOR 1.5
    x = O.nrc_inputs((0, 0, 0), (1, 1, 1), (0.5, 0.5, 0.5), (0, 0, 1), (0, 0, 1),
                     scenes.material(base_color=(0.3, 0.4, 0.5), specular_weight=1.0))
    assert abs(x[11] - 0.04) < 1e-15


def test_factorised_cache_query_multiplies_by_the_factor(O):
    """The box seen through a cache answering c at vertex 0: every path that
    hits a Lambertian wall first carries c * rho (the walls' specular input is
    0; emission at vertex 0 aside, the light's own albedo factor is 0)."""
    sc = scenes.cornell(width=16, height=16)
    os_ = O.OracleScene(sc)
    r = os_.render(2, 4, per_sample=True, nrc_weights=_constant_cache(0.5), nrc_bounce=0, nrc_factor=True)
    rp = os_.render(2, 4, per_sample=True, nrc_weights=_constant_cache(0.5), nrc_bounce=0)
    v, vp = r["per_sample"].reshape(-1, 3), rp["per_sample"].reshape(-1, 3)
    alb = sc.materials[:7, 1:4].astype(np.float64)
    ok = 0
    for a, b in zip(v, vp):
        if np.allclose(b, 0.5, rtol=1e-12):  # a wall: the plain query gives 0.5 exactly
            rho = a / 0.5
            assert np.any(np.all(np.isclose(alb, rho, rtol=1e-6, atol=1e-7), axis=1)), rho
            ok += 1
    assert ok > 100


# ------------------------------------------------------- adaptive termination --

def test_spread_termination_limits(O):
    """Spread heuristic of the cited method: any non-delta bounce adds spread, so
    with a vanishing threshold every path ends in the cache at vertex 1 (as with
    a fixed query at vertex 1); with a huge threshold none does before the
    fixed query vertex; in between, the share ending early falls as the
    threshold grows."""
    sc = scenes.cornell(width=16, height=16)
    os_ = O.OracleScene(sc)
    w = N.init_weights(3, O.uniform)
    kw = dict(per_sample=True, nrc_weights=w, nrc_bf16=False)
    r1 = os_.render(2, 5, nrc_bounce=1, **kw)
    r2 = os_.render(2, 5, nrc_bounce=2, **kw)
    tiny = os_.render(2, 5, nrc_bounce=2, spread_c=1e-30, **kw)
    huge = os_.render(2, 5, nrc_bounce=2, spread_c=1e30, **kw)
    assert np.array_equal(tiny["per_sample"], r1["per_sample"]) and np.array_equal(tiny["sigs"], r1["sigs"])
    assert np.array_equal(huge["per_sample"], r2["per_sample"]) and np.array_equal(huge["sigs"], r2["sigs"])
    assert not np.array_equal(r1["sigs"], r2["sigs"])
    early = []
    for c in (1e-3, 1e-2, 1e-1, 1.0, 10.0, 100.0):
        r = os_.render(2, 5, nrc_bounce=2, spread_c=c, **kw)
        early.append(float((r["sigs"] == r1["sigs"]).mean()))
    assert all(a >= b for a, b in zip(early, early[1:])), early
    assert early[0] > 0.9 and early[-1] < early[0]


def test_spread_of_a_delta_bounce_is_zero(O):
    """A mirror floor (metal, roughness 0): a path whose first bounce is the
    mirror's delta reflection has no spread at vertex 1 and does not end there
    even with a vanishing threshold; paths that scatter diffusely first do."""
    import dataclasses
    sc = scenes.cornell(width=16, height=16)
    m = sc.materials.copy()
    m[0] = scenes.material(base_metalness=1.0, base_color=(0.9, 0.9, 0.9), specular_roughness=0.0)
    sc = dataclasses.replace(sc, materials=m)
    os_ = O.OracleScene(sc)
    w = N.init_weights(4, O.uniform)
    kw = dict(per_sample=True, nrc_weights=w)
    r1 = os_.render(2, 5, nrc_bounce=1, **kw)
    r2 = os_.render(2, 5, nrc_bounce=2, **kw)
    tiny = os_.render(2, 5, nrc_bounce=2, spread_c=1e-30, **kw)
    as1 = tiny["sigs"] == r1["sigs"]
    as2 = tiny["sigs"] == r2["sigs"]
    differ = r1["sigs"] != r2["sigs"]
    assert np.all(as1 | as2)
    # among paths where the fixed vertex matters, the mirror's (bottom rows) keep going to vertex 2
    bottom = np.zeros_like(as1)
    bottom[12:] = True
    assert as2[differ & bottom].mean() > 0.5 and as1[differ & ~bottom].mean() > 0.9
