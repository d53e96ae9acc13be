"""GPU parity of the radiance cache (future work named in Sec. 6.1) against the oracle.

* Network: the matrix-core forward and gradient against the FP64 numpy
  oracle that rounds the same operands to bfloat16.  Emulating the GPU's
  FP32 sums in numpy puts 99.9% of outputs within 1e-5 of |y| + rms(y) and
  the worst at 2e-3 on 4099 rows, 1.5e-2 on the 32,933 rows of the
  full-size check (a bfloat16 rounding flip of a hidden activation carried
  to the output); the gates are 1e-4 for 99.9% and 5e-3 (3e-2 on the
  full-size rows) for all.
* Adam: two steps on batches drawn by the documented Philox rule, against
  the oracle's Adam on the oracle's own gradients.
* Paths: render paths that end in the cache carry the same event signature
  and radiance as the oracle's; training records of the frame's training
  paths equal the oracle's, path by path.
* Closed form: a network that outputs 1 on the white furnace gives 1.
* The frame loop learns: the loss on held-out records falls.
* Frames of one call, which overlap on two path sets, give bitwise the sums
  and weights of one call per frame.
"""
import math

import numpy as np
import pytest

from oracle import nrc_np as N
from paper_2407_19977_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19977_amd import pt
    return pt


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to("cuda:0")


def _inputs(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    return r.uniform(0, 1, (n, 12)).astype(np.float32)


def _weights(O, seed):
    """He-uniform weights of the oracle, rounded to the FP32 the GPU keeps."""
    return N.init_weights(seed, O.uniform).astype(np.float32)


_scenes = {}


def _cache_scene(P, O, key, make, cfg):
    if key not in _scenes:
        sc = make()
        _say(f"[scene] {key}: {sc.n_triangles} triangles")
        _scenes[key] = (sc, P.scene_from(sc, device=0), O.OracleScene(sc))
    sc, s, os_ = _scenes[key]
    s.set_radiance_cache(cfg)
    return sc, s, os_


def _net_scene(P, O):
    return _cache_scene(P, O, "cornell", scenes.cornell, P.cache_config())


# ------------------------------------------------------------------ network --

@pytest.mark.parametrize("n", [1, 17, 4099])
def test_forward_matches_bf16_oracle(P, O, n):
    _say(f"[nrc forward] n={n}")
    _, s, _ = _net_scene(P, O)
    w = _weights(O, 7)
    s.nrc_set_weights(_dev(w))
    X = _inputs(n, 1)
    y = torch.empty((n, 3), dtype=torch.float32, device="cuda:0")
    s.nrc_forward(_dev(X), y)
    y = y.cpu().numpy().astype(np.float64)
    ref, _ = N.forward(w.astype(np.float64), X.astype(np.float64), use_bf16=True)
    scale = math.sqrt(float((ref ** 2).mean())) + 1e-12
    rel = np.abs(y - ref) / (np.abs(ref) + scale)
    _say(f"[nrc forward] n={n} rel err max {rel.max():.2e} p99.9 {np.quantile(rel, 0.999):.2e}")
    assert np.all(np.isfinite(y))
    assert np.quantile(rel, 0.999) <= 1e-4
    assert rel.max() <= 5e-3


def test_forward_full_size_sampled(P, O):
    """A full frame's worth of queries (2^21 + 37: every tile plus a ragged
    tail) in one launch, checked on 2^15 sampled rows (the first and last
    tiles included) against the bf16-rounding oracle."""
    n = (1 << 21) + 37
    _say(f"[nrc forward] n={n} (sampled check)")
    _, s, _ = _net_scene(P, O)
    w = _weights(O, 13)
    s.nrc_set_weights(_dev(w))
    X = _inputs(n, 3)
    y = torch.empty((n, 3), dtype=torch.float32, device="cuda:0")
    s.nrc_forward(_dev(X), y)
    y = y.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(y))
    r = np.random.Generator(np.random.PCG64(14))
    sel = np.unique(np.concatenate([np.arange(64), np.arange(n - 101, n), r.choice(n, 1 << 15, replace=False)]))
    ref, _ = N.forward(w.astype(np.float64), X[sel].astype(np.float64), use_bf16=True)
    scale = math.sqrt(float((ref ** 2).mean())) + 1e-12
    rel = np.abs(y[sel] - ref) / (np.abs(ref) + scale)
    _say(f"[nrc forward] n={n}: {len(sel)} rows, rel err max {rel.max():.2e} p99.9 {np.quantile(rel, 0.999):.2e}")
    assert np.quantile(rel, 0.999) <= 1e-4
    # FP32 sums emulated in numpy on these same rows flip a bfloat16 rounding in 7 of
    # 32,933 rows; the worst of them reaches 1.5e-2 at the output (one flipped hidden
    # activation carried through the remaining layers), hence 3e-2 for the maximum here
    assert rel.max() <= 3e-2


def test_forward_of_permutation_network_is_exact(P, O):
    """Permutation matrices move bfloat16 features without arithmetic: the
    output is the encoded feature the index bookkeeping names, rounded to bf16."""
    _, s, _ = _net_scene(P, O)
    r = np.random.Generator(np.random.PCG64(4))
    sig = [r.permutation(64) for _ in range(5)]
    mats = []
    for sg in sig:
        M = np.zeros((64, 64))
        M[np.arange(64), sg] = 1.0
        mats.append(M)
    pick = r.choice(64, 3, replace=False)
    W5 = np.zeros((3, 64))
    W5[np.arange(3), pick] = 1.0
    w = N.pack(mats + [W5]).astype(np.float32)
    s.nrc_set_weights(_dev(w))
    X = _inputs(300, 2)
    y = torch.empty((300, 3), dtype=torch.float32, device="cuda:0")
    s.nrc_forward(_dev(X), y)
    y = y.cpu().numpy().astype(np.float64)
    idx = np.arange(64)
    for sg in reversed(sig):
        idx = sg[idx]
    F = N.encode(X.astype(np.float64))
    expect = np.maximum(N.bf16(F[:, idx[pick]]), 0.0)
    # the GPU evaluates sin / cos in FP32: allow one bf16 step of the feature
    err = np.abs(y - expect)
    assert np.all(err <= 2.0 ** -7 * np.maximum(np.abs(expect), 2.0 ** -20) + 1e-6), err.max()
    assert np.mean(err == 0) > 0.97


def test_gradient_matches_bf16_oracle_and_repeats_bitwise(P, O):
    _say("[nrc gradient] n=3001")
    _, s, _ = _net_scene(P, O)
    w = _weights(O, 11)
    s.nrc_set_weights(_dev(w))
    n = 3001
    X = _inputs(n, 5)
    T = np.random.Generator(np.random.PCG64(6)).uniform(0, 2, (n, 3)).astype(np.float32)
    g1 = torch.empty(P.NRC_PARAMS, dtype=torch.float32, device="cuda:0")
    g2 = torch.empty_like(g1)
    loss1 = s.nrc_gradient(_dev(X), _dev(T), g1)
    loss2 = s.nrc_gradient(_dev(X), _dev(T), g2)
    assert torch.equal(g1, g2) and loss1 == loss2
    g = g1.cpu().numpy().astype(np.float64)
    lref, gref = N.gradient(w.astype(np.float64), X.astype(np.float64), T.astype(np.float64), use_bf16=True)
    _say(f"[nrc gradient] loss gpu {loss1:.6f} oracle {lref:.6f}")
    assert abs(loss1 - lref) <= 1e-3 * lref
    for l in range(6):
        sl = slice(4096 * l, 4096 * (l + 1)) if l < 5 else slice(20480, None)
        e = np.linalg.norm(g[sl] - gref[sl]) / np.linalg.norm(gref[sl])
        _say(f"[nrc gradient] layer {l} rel err {e:.2e}")
        assert e <= 1e-2


def _batch(O, seed, frame, step, n, B):
    """Record indices of the batch of a step: floor(m n / 2^24), m the top 24
    bits of Philox word step % 4 at (j, 2^31 + frame, 0x4E5253, step / 4)."""
    m = np.array([round(O.uniform(seed, j, 0x80000000 + frame, 0x4E5253, step) * 16777216.0) for j in range(B)],
                 dtype=np.int64)
    return (m * n) >> 24


def test_two_adam_steps_match_oracle(P, O):
    _say("[nrc adam] 2 steps, batch 2048 from 5000 records")
    sc, s, _ = _cache_scene(P, O, "cornell", scenes.cornell,
                            P.cache_config(batch_size=2048, steps_per_frame=2, ema_decay=0.99))
    w = _weights(O, 3)
    s.nrc_set_weights(_dev(w))
    n, seed, frame = 5000, 9, 6
    X = _inputs(n, 7)
    T = np.random.Generator(np.random.PCG64(8)).uniform(0, 2, (n, 3)).astype(np.float32)
    s.nrc_train(_dev(X), _dev(T), frame, seed)
    wg = torch.empty(P.NRC_PARAMS, dtype=torch.float32, device="cuda:0")
    mg, vg = torch.empty_like(wg), torch.empty_like(wg)
    step = s.nrc_get_weights(wg, mg, vg)
    assert step == 2
    wr = w.astype(np.float64)
    m = np.zeros_like(wr)
    v = np.zeros_like(wr)
    g_steps = []
    for k in range(2):
        idx = _batch(O, seed, frame, k, n, 2048)
        _, g = N.gradient(wr, X[idx].astype(np.float64), T[idx].astype(np.float64), use_bf16=True)
        g_steps.append(g)
        wr, m, v = N.adam(wr, m, v, g, k + 1)
    dw = np.abs(wg.cpu().numpy() - wr)
    lr = 1e-3
    _say(f"[nrc adam] |w_gpu - w_ref| / lr: p99 {np.quantile(dw, 0.99) / lr:.3e} max {dw.max() / lr:.3e}")
    assert np.quantile(dw, 0.99) <= 0.05 * lr
    # Where the gradient is well above the bfloat16 noise of its layer (both
    # steps' |g| above 1e-2 of the layer's rms gradient, and the bias-corrected
    # first moment not cancelled, |m_hat| >= 0.1 sqrt(v_hat)), the update is
    # well conditioned and the GPU's weights follow the oracle's to 0.05 lr.
    # Elsewhere Adam's normalisation turns a bfloat16-sized gradient
    # difference into a change of the step's sign, bounded only by 2 lr.
    layer_rms = np.zeros_like(wr)
    for l in range(6):
        sl = slice(4096 * l, 4096 * (l + 1)) if l < 5 else slice(20480, None)
        layer_rms[sl] = np.sqrt(np.mean(g_steps[0][sl] ** 2))
    mh = m / (1 - 0.9 ** 2)
    vh = v / (1 - 0.99 ** 2)
    good = (np.abs(g_steps[0]) > 1e-2 * layer_rms) & (np.abs(g_steps[1]) > 1e-2 * layer_rms) & \
        (np.abs(mh) >= 0.1 * np.sqrt(vh))
    _say(f"[nrc adam] well-conditioned weights {int(good.sum())} / {good.size}: max |dw| / lr "
         f"{dw[good].max() / lr:.3e}; all weights max {dw.max() / lr:.3e}")
    assert good.sum() > 0.5 * good.size
    assert dw[good].max() <= 0.05 * lr
    em = np.linalg.norm(mg.cpu().numpy() - m) / np.linalg.norm(m)
    assert em <= 2e-2, em
    # inference weights: the bias-corrected moving average (decay 0.99) of the two steps' weights
    wi = torch.empty_like(wg)
    s.nrc_get_inference_weights(wi)
    wr1 = w.astype(np.float64)
    e = np.zeros_like(wr1)
    mm, vv = np.zeros_like(wr1), np.zeros_like(wr1)
    for k in range(2):
        wr1, mm, vv = N.adam(wr1, mm, vv, g_steps[k], k + 1)
        e = N.ema_update(e, wr1, 0.99)
    wi_ref = N.ema_weights(e, 2, 0.99, wr1)
    di = np.abs(wi.cpu().numpy() - wi_ref)
    _say(f"[nrc adam] inference weights |wi_gpu - wi_ref| / lr: p99 {np.quantile(di, 0.99) / lr:.3e} "
         f"max {di.max() / lr:.3e}")
    assert np.quantile(di, 0.99) <= 0.05 * lr
    assert di[good].max() <= 0.05 * lr
    # the average of two steps is not the latest weights
    assert np.abs(wi.cpu().numpy() - wg.cpu().numpy()).max() > 0.1 * lr


def test_inference_weights_without_moving_average_are_the_weights(P, O):
    """ema_decay 0: after Adam steps the cache queries use the weights themselves."""
    sc, s, _ = _cache_scene(P, O, "cornell", scenes.cornell,
                            P.cache_config(batch_size=512, steps_per_frame=3, ema_decay=0.0))
    s.nrc_set_weights(_dev(_weights(O, 4)))
    n = 700
    X = _inputs(20000, 17)[:n]
    T = np.random.Generator(np.random.PCG64(18)).uniform(0, 2, (n, 3)).astype(np.float32)
    s.nrc_train(_dev(X), _dev(T), 2, 5)
    wg = torch.empty(P.NRC_PARAMS, dtype=torch.float32, device="cuda:0")
    wi = torch.empty_like(wg)
    assert s.nrc_get_weights(wg) == 3
    s.nrc_get_inference_weights(wi)
    assert torch.equal(wg, wi)
    # and the forward call answers with them (20,000 queries: the bfloat16 flip rate of FP32 sums,
    # about 2 rows in 10^4, is then resolved by the 99.9th percentile)
    Xq = _inputs(20000, 19)
    y = torch.empty((20000, 3), dtype=torch.float32, device="cuda:0")
    s.nrc_forward(_dev(Xq), y)
    ref, _ = N.forward(wg.cpu().numpy().astype(np.float64), Xq.astype(np.float64), use_bf16=True)
    scale = math.sqrt(float((ref ** 2).mean()))
    rel = np.abs(y.cpu().numpy() - ref) / (np.abs(ref) + scale)
    assert np.quantile(rel, 0.999) <= 1e-4 and rel.max() <= 3e-2


# -------------------------------------------------------------------- paths --

def _constant_cache(value):
    mats = [np.zeros((64, 64)) for _ in range(5)]
    for M in mats:
        M[60, 60] = 1.0
    W5 = np.zeros((3, 64))
    W5[:, 60] = value
    return N.pack(mats + [W5]).astype(np.float32)


def test_unit_cache_on_white_furnace_gives_one(P, O):
    """Convex white object under a sky of 1, cache returning 1 from the first
    hit: every path carries exactly 1 (up to FP32 rounding of beta)."""
    _say("[nrc furnace] unit cache at vertex 0")
    sc = scenes.furnace("sphere", width=16, height=16)
    s = P.scene_from(sc, device=0)
    s.set_radiance_cache(P.cache_config(query_bounce=0, factorize=0))
    s.nrc_set_weights(_dev(_constant_cache(1.0)))
    per = torch.empty((16, 16, 4, 3), dtype=torch.float32, device="cuda:0")
    sig = torch.empty((16, 16, 4), dtype=torch.int64, device="cuda:0")
    s.render_debug(sc.camera, 0, 0, 16, 16, 0, 4, 5, 0, per, sig)
    v = per.cpu().numpy()
    assert np.allclose(v, 1.0, atol=1e-6, rtol=0)
    s.close()


def test_cache_terminated_paths_match_oracle(P, O):
    _say("[nrc paths] box scene 48x48 crop, 4 spp, depth 6, cache at vertex 2")
    sc, s, os_ = _cache_scene(P, O, "cornell", scenes.cornell,
                              P.cache_config(query_bounce=2, spread_c=0.0, factorize=0))
    w = _weights(O, 21)
    s.nrc_set_weights(_dev(w))
    crop, spp, depth = (40, 40, 48, 48), 4, 6
    x0, y0, cw, ch = crop
    per = torch.empty((ch, cw, spp, 3), dtype=torch.float32, device="cuda:0")
    sig = torch.empty((ch, cw, spp), dtype=torch.int64, device="cuda:0")
    s.render_debug(sc.camera, x0, y0, cw, ch, 0, spp, depth, 0, per, sig)
    g = per.cpu().numpy().astype(np.float64)
    gs = sig.cpu().numpy().view(np.uint64)
    ref = os_.render(spp, depth, crop=crop, per_sample=True, nrc_weights=w.astype(np.float64), nrc_bounce=2,
                     nrc_bf16=True)
    match = gs == ref["sigs"]
    frac = float(match.mean())
    o = ref["per_sample"]
    floor = 1e-6 * max(1.0, float(o.mean()))
    rel = (np.abs(g - o).max(-1) / (np.abs(o).max(-1) + floor))[match]
    bias = float((g - o)[match].mean() / o[match].mean())
    _say(f"[nrc paths] identical {frac * 100:.3f}%  rel err p99 {np.quantile(rel, 0.99):.2e} "
         f"p99.9 {np.quantile(rel, 0.999):.2e} max {rel.max():.2e}  mean bias {bias:.2e}")
    assert frac >= 0.999
    # The cache inputs come from FP32 hit points and directions.  In the FP64
    # oracle itself, moving the 12 inputs by 1e-7 (FP32 rounding) flips
    # bfloat16 roundings of the high-frequency features and moves the output
    # of this random (untrained, chaotic) network by up to a few per cent;
    # such flips are rare on the GPU's paths (measured p99 2e-6, p99.9 9e-3).
    # The gates hold the 99th percentile to 1e-4, allow at most 2 in 10^4
    # paths (2 in any case) beyond 5e-2, and the flips must not bias the mean.
    assert np.quantile(rel, 0.99) <= 1e-4
    assert (rel > 5e-2).sum() <= max(2, int(2e-4 * rel.size)), np.sort(rel)[-5:]
    assert abs(bias) <= 1e-3
    assert np.isfinite(g).all()


def test_training_records_match_oracle(P, O):
    _say("[nrc records] box scene 32x32, 1024 training paths, depth 5, frame 3")
    sc0 = scenes.cornell(width=32, height=32)
    sc, s, os_ = _cache_scene(P, O, "cornell32", lambda: sc0,
                              P.cache_config(train_paths=1024, train_end_bounce=-1, factorize=0))
    depth, frame, seed = 5, 3, 0
    cap = 1024 * depth
    X = torch.empty((cap, 12), dtype=torch.float32, device="cuda:0")
    T = torch.empty((cap, 3), dtype=torch.float32, device="cuda:0")
    off = torch.empty(1024, dtype=torch.int32, device="cuda:0")
    n = s.nrc_training_records(sc.camera, frame, depth, seed, X, T, off)
    X, T, off = X.cpu().numpy()[:n].astype(np.float64), T.cpu().numpy()[:n].astype(np.float64), off.cpu().numpy()
    WH = 32 * 32
    stride = max(1, WH // 1024)
    m = round(O.uniform(seed, 0, 0x80000000 + frame, 0x4F4646, 0) * 16777216.0)
    o_f = (m * WH) >> 24
    good = 0
    total_ref = 0
    for k in range(1024):
        pix = (k * stride + o_f) % WH
        xr, tr = os_.training_records(pix % 32, pix // 32, 0x80000000 + frame, depth, seed)
        total_ref += len(xr)
        a, b = int(off[k]), int(off[k + 1]) if k + 1 < 1024 else n
        if b - a != len(xr):
            continue
        if len(xr) == 0:
            good += 1
            continue
        dx = np.abs(X[a:b] - xr)
        dt = np.abs(T[a:b] - tr)
        if np.all(dx <= 1e-4) and np.all(dt <= 1e-3 * np.abs(tr) + 1e-5 * max(1.0, float(np.abs(tr).max()))):
            good += 1
    _say(f"[nrc records] {n} records (oracle {total_ref}), paths identical {good}/1024")
    assert good >= 0.99 * 1024
    assert abs(n - total_ref) <= 0.02 * total_ref


@pytest.mark.parametrize("train_end,factorize", [(2, 0), (2, 1), (-1, 1)])
def test_self_trained_and_factorised_records_match_oracle(P, O, train_end, factorize):
    """Training records with the refinements of the cited cache method: training
    paths that end in the cache at vertex 2 (self-training: the cache's answer
    there, under given weights, joins the radiance of the path's earlier
    vertices) and targets divided by the reflectance factor."""
    _say(f"[nrc records] box 32x32, 1024 training paths, depth 5, train_end {train_end}, factorize {factorize}")
    sc0 = scenes.cornell(width=32, height=32)
    cfg = P.cache_config(train_paths=1024, train_end_bounce=train_end, factorize=factorize)
    sc, s, os_ = _cache_scene(P, O, "cornell32", lambda: sc0, cfg)
    w = _weights(O, 31)
    s.nrc_set_weights(_dev(w))  # weights given: the cache is in use, self-training on
    depth, frame, seed = 5, 4, 0
    cap = 1024 * depth
    X = torch.empty((cap, 12), dtype=torch.float32, device="cuda:0")
    T = torch.empty((cap, 3), dtype=torch.float32, device="cuda:0")
    off = torch.empty(1024, dtype=torch.int32, device="cuda:0")
    n = s.nrc_training_records(sc.camera, frame, depth, seed, X, T, off)
    X, T, off = X.cpu().numpy()[:n].astype(np.float64), T.cpu().numpy()[:n].astype(np.float64), off.cpu().numpy()
    WH = 32 * 32
    stride = max(1, WH // 1024)
    m = round(O.uniform(seed, 0, 0x80000000 + frame, 0x4F4646, 0) * 16777216.0)
    o_f = (m * WH) >> 24
    good = total_ref = 0
    for k in range(1024):
        pix = (k * stride + o_f) % WH
        xr, tr = os_.training_records(pix % 32, pix // 32, 0x80000000 + frame, depth, seed,
                                      nrc_weights=w.astype(np.float64), train_end=train_end, nrc_bf16=True,
                                      factorize=bool(factorize))
        total_ref += len(xr)
        a, b = int(off[k]), int(off[k + 1]) if k + 1 < 1024 else n
        if b - a != len(xr):
            continue
        if len(xr) == 0:
            good += 1
            continue
        if train_end >= 0:
            assert len(xr) <= train_end
        dx = np.abs(X[a:b] - xr)
        dt = np.abs(T[a:b] - tr)
        if np.all(dx <= 1e-4) and np.all(dt <= 1e-3 * np.abs(tr) + 1e-5 * max(1.0, float(np.abs(tr).max()))):
            good += 1
    _say(f"[nrc records] {n} records (oracle {total_ref}), paths identical {good}/1024")
    assert good >= 0.98 * 1024
    assert abs(n - total_ref) <= 0.02 * total_ref


def test_factorised_cache_paths_match_oracle(P, O):
    _say("[nrc paths] box 48x48 crop, 4 spp, depth 6, factorised cache at vertex 1")
    sc, s, os_ = _cache_scene(P, O, "cornell", scenes.cornell,
                              P.cache_config(query_bounce=1, spread_c=0.0, factorize=1))
    w = _weights(O, 22)
    s.nrc_set_weights(_dev(w))
    crop, spp, depth = (40, 40, 48, 48), 4, 6
    x0, y0, cw, ch = crop
    per = torch.empty((ch, cw, spp, 3), dtype=torch.float32, device="cuda:0")
    sig = torch.empty((ch, cw, spp), dtype=torch.int64, device="cuda:0")
    s.render_debug(sc.camera, x0, y0, cw, ch, 0, spp, depth, 0, per, sig)
    g = per.cpu().numpy().astype(np.float64)
    gs = sig.cpu().numpy().view(np.uint64)
    ref = os_.render(spp, depth, crop=crop, per_sample=True, nrc_weights=w.astype(np.float64), nrc_bounce=1,
                     nrc_bf16=True, nrc_factor=True)
    match = gs == ref["sigs"]
    o = ref["per_sample"]
    floor = 1e-6 * max(1.0, float(o.mean()))
    rel = (np.abs(g - o).max(-1) / (np.abs(o).max(-1) + floor))[match]
    bias = float((g - o)[match].mean() / o[match].mean())
    _say(f"[nrc paths] factorised: identical {match.mean() * 100:.3f}%  rel err p99 {np.quantile(rel, 0.99):.2e} "
         f"max {rel.max():.2e}  mean bias {bias:.2e}")
    assert match.mean() >= 0.999
    assert np.quantile(rel, 0.99) <= 1e-4   # the same gates as the unfactorised paths
    assert rel.max() <= 5e-2
    assert abs(bias) <= 1e-3


@pytest.mark.parametrize("which", ["cornell", "zoo"])
def test_adaptive_termination_paths_match_oracle(P, O, which):
    """Paths end in the cache where their spread first exceeds 0.01 of the
    primary footprint (delta bounces add none), at vertex 3 at the latest."""
    _say(f"[nrc paths] {which}: adaptive termination, spread threshold 0.01, query vertex 3 at the latest")
    make = scenes.cornell if which == "cornell" else scenes.material_zoo
    sc, s, os_ = _cache_scene(P, O, which, make, P.cache_config(query_bounce=3, spread_c=0.01, factorize=0))
    # A random network is chaotic in the high-frequency position features: the
    # GPU's FP32 hit points flip their bfloat16 roundings now and then and move
    # the answer by up to a few per cent, which dominates paths that end at
    # vertex 1.  With the inputs of frequencies 4 pi and up switched off, the
    # cache answer is smooth and the per-path gates are those of the plain tracer.
    w = _weights(O, 23)
    W0 = w[:4096].reshape(64, 64)
    for f in range(36):
        if ((f % 12) >> 1) >= 2:
            W0[:, f] = 0.0
    s.nrc_set_weights(_dev(w))
    crop, spp, depth = ((40, 40, 48, 48) if which == "cornell" else (24, 24, 48, 48)), 4, 6
    x0, y0, cw, ch = crop
    per = torch.empty((ch, cw, spp, 3), dtype=torch.float32, device="cuda:0")
    sig = torch.empty((ch, cw, spp), dtype=torch.int64, device="cuda:0")
    s.render_debug(sc.camera, x0, y0, cw, ch, 0, spp, depth, 0, per, sig)
    g = per.cpu().numpy().astype(np.float64)
    gs = sig.cpu().numpy().view(np.uint64)
    ref = os_.render(spp, depth, crop=crop, per_sample=True, nrc_weights=w.astype(np.float64), nrc_bounce=3,
                     nrc_bf16=True, spread_c=0.01)
    fixed = os_.render(spp, depth, crop=crop, per_sample=True, nrc_weights=w.astype(np.float64), nrc_bounce=3,
                       nrc_bf16=True)
    match = gs == ref["sigs"]
    o = ref["per_sample"]
    floor = 1e-6 * max(1.0, float(o.mean()))
    rel = (np.abs(g - o).max(-1) / (np.abs(o).max(-1) + floor))[match]
    early = float((ref["sigs"] != fixed["sigs"]).mean())
    _say(f"[nrc paths] {which}: identical {match.mean() * 100:.3f}%, ended before vertex 3 {early * 100:.1f}%, "
         f"rel err p99 {np.quantile(rel, 0.99):.2e} max {rel.max():.2e}")
    assert early > 0.2  # the heuristic ends a good share of the paths early
    assert match.mean() >= 0.99
    assert np.quantile(rel, 0.99) <= 1e-4
    # Directions within FP32 rounding of the poles of the spherical inputs (the floor's normal,
    # vertical bounces) have an azimuth decided by rounding noise; such a query may answer
    # differently on the two sides.  At most 2 paths in 10^4 (and 2 in any case) may exceed 5e-2.
    assert (rel > 5e-2).sum() <= max(2, int(2e-4 * rel.size)), np.sort(rel)[-5:]


@pytest.mark.parametrize("spread", [0.0, 0.01])
def test_tail_kernel_ends_paths_in_the_cache(P, O, spread):
    """With the persistent tail kernel taking over at bounce 1, before the
    query vertex, the tail ends the paths in the cache (fixed vertex 2, or
    adaptively) and queues their queries; the query kernel then runs after it.
    The paths equal the oracle's as in the wavefront."""
    _say(f"[nrc paths] box scene, tail kernel from bounce 1, cache at vertex 2, spread {spread}")
    sc, s, os_ = _cache_scene(P, O, "cornell", scenes.cornell,
                              P.cache_config(query_bounce=2, spread_c=spread, factorize=0))
    w = _weights(O, 29)
    W0 = w[:4096].reshape(64, 64)
    for f in range(36):  # a smooth answer: the inputs of frequencies 4 pi and up switched off
        if ((f % 12) >> 1) >= 2:
            W0[:, f] = 0.0
    s.nrc_set_weights(_dev(w))
    crop, spp, depth = (40, 40, 48, 48), 4, 6
    x0, y0, cw, ch = crop
    per = torch.empty((ch, cw, spp, 3), dtype=torch.float32, device="cuda:0")
    sig = torch.empty((ch, cw, spp), dtype=torch.int64, device="cuda:0")
    s.set_tail(1, 1.0)
    try:
        s.reset_stats()
        s.render_debug(sc.camera, x0, y0, cw, ch, 0, spp, depth, 0, per, sig)
        st = s.stats()
    finally:
        s.set_tail()
    assert st["tail_extension_rays"] > 0 and st["cache_queries"] > 0
    g = per.cpu().numpy().astype(np.float64)
    gs = sig.cpu().numpy().view(np.uint64)
    ref = os_.render(spp, depth, crop=crop, per_sample=True, nrc_weights=w.astype(np.float64), nrc_bounce=2,
                     nrc_bf16=True, spread_c=spread)
    match = gs == ref["sigs"]
    o = ref["per_sample"]
    floor = 1e-6 * max(1.0, float(o.mean()))
    rel = (np.abs(g - o).max(-1) / (np.abs(o).max(-1) + floor))[match]
    _say(f"[nrc paths] tail from bounce 1, spread {spread}: identical {match.mean() * 100:.3f}%, "
         f"queries {st['cache_queries']}, rel err p99 {np.quantile(rel, 0.99):.2e} max {rel.max():.2e}")
    assert match.mean() >= 0.99
    assert np.quantile(rel, 0.99) <= 1e-4
    assert (rel > 5e-2).sum() <= max(2, int(2e-4 * rel.size)), np.sort(rel)[-5:]


# --------------------------------------------------------------- frame loop --

def test_frame_loop_learns_and_counts_steps(P, O):
    _say("[nrc frames] box scene 64x64, 24 frames")
    sc0 = scenes.cornell(width=64, height=64)
    sc, s, os_ = _cache_scene(P, O, "cornell64", lambda: sc0,
                              P.cache_config(train_paths=4096, batch_size=4096, steps_per_frame=4))
    depth, seed = 5, 0
    cap = 4096 * depth
    Xh = torch.empty((cap, 12), dtype=torch.float32, device="cuda:0")
    Th = torch.empty((cap, 3), dtype=torch.float32, device="cuda:0")
    nh = s.nrc_training_records(sc.camera, 1000, depth, seed, Xh, Th)   # held-out frame
    assert nh > 1000
    Xh, Th = Xh[:nh].contiguous(), Th[:nh].contiguous()
    grad = torch.empty(P.NRC_PARAMS, dtype=torch.float32, device="cuda:0")
    loss0 = s.nrc_gradient(Xh, Th, grad)
    s.reset_accumulation()
    s.accumulate(sc.camera, 0, 24, depth, seed)
    step = s.nrc_get_weights()
    assert step == 24 * 4
    loss1 = s.nrc_gradient(Xh, Th, grad)
    _say(f"[nrc frames] held-out loss {loss0:.4f} -> {loss1:.4f}")
    assert loss1 < 0.7 * loss0
    out = torch.empty((64, 64, 3), dtype=torch.float32, device="cuda:0")
    s.resolve(out)
    img = out.cpu().numpy()
    assert np.isfinite(img).all() and img.mean() > 0
    s.set_radiance_cache(None)


def test_overlapped_frames_equal_frame_by_frame(P, O):
    """Frames of one call overlap (a frame's training beside the next frame's
    bounces, on two path sets); the FP64 sums, weights, Adam moments and step
    count must be bitwise those of one call per frame.  64x64 with 512
    training paths, so the tail takes the training paths over without a
    host read of the path count (512 <= 1/8 of 4096 + 512 slots)."""
    _say("[nrc overlap] box scene 64x64, 6 frames, 512 training paths")
    sc = scenes.cornell(width=64, height=64)
    cfg = P.cache_config(train_paths=512, batch_size=512, steps_per_frame=2)
    _, s, _ = _cache_scene(P, O, "cornell64b", lambda: sc, cfg)
    depth, seed, frames = 5, 3, 6
    out = torch.empty((64, 64, 3), dtype=torch.float32, device="cuda:0")
    results = []
    for one_call in (True, False):
        s.set_radiance_cache(cfg)
        s.reset_accumulation()
        s.reset_stats()
        if one_call:
            s.accumulate(sc.camera, 0, frames, depth, seed)
        else:
            for k in range(frames):
                s.accumulate(sc.camera, k, 1, depth, seed)
        acc = torch.empty((64, 64, 3), dtype=torch.float64, device="cuda:0")
        s.resolve(out, acc)
        w = torch.empty(P.NRC_PARAMS, dtype=torch.float32, device="cuda:0")
        m, v = torch.empty_like(w), torch.empty_like(w)
        step = s.nrc_get_weights(w, m, v)
        st = s.stats()
        results.append((acc.cpu().numpy(), w.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), step,
                        st["cache_records"], st["cache_queries"]))
    a, b = results
    assert a[4] == b[4] == frames * 2
    assert a[5] == b[5] > 0 and a[6] == b[6] > 0
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    s.set_radiance_cache(None)


def test_cache_api_errors(P, O):
    sc = scenes.cornell(width=8, height=8)
    s = P.scene_from(sc, device=0)
    w = torch.zeros(P.NRC_PARAMS, dtype=torch.float32, device="cuda:0")
    with pytest.raises(P.PtError) as e:
        s.nrc_set_weights(w)
    assert e.value.status == -5
    with pytest.raises(P.PtError) as e:
        s.set_radiance_cache(P.cache_config(batch_size=0))
    assert e.value.status == -1
    with pytest.raises(P.PtError) as e:
        s.set_radiance_cache(P.cache_config(beta2=1.0))
    assert e.value.status == -1
    s.set_radiance_cache(P.cache_config())
    with pytest.raises(P.PtError) as e:
        s.nrc_set_weights(w[:100])
    assert e.value.status == -1
    s.close()


def test_trained_cache_lowers_rmse_at_equal_samples(P, O):
    """What the trained network gains: the box scene with bright walls (albedo
    0.85, so much of the light arrives after the third vertex), 64x64, depth
    12, 64 frames of 1 spp with the cache (query at vertex 2, trained online
    from frame 0 on 512 training paths per frame) against 64 frames of the
    plain tracer, both against a 4096-spp plain reference with an independent
    seed.  The cached image has the lower RMSE at equal samples, and the
    lower RMSE^2 x rays traced (training rays included)."""
    import dataclasses
    _say("[nrc gain] bright box 64x64, depth 12, 64 frames, reference 4096 spp")
    sc = scenes.cornell(width=64, height=64)
    m = sc.materials.copy()
    m[m[:, 23] == 0, 1:4] = 0.85
    sc = dataclasses.replace(sc, materials=m)
    s = P.scene_from(sc, device=0)
    cam, depth = sc.camera, 12
    out = torch.empty((64, 64, 3), dtype=torch.float32, device="cuda:0")
    acc = torch.empty((64, 64, 3), dtype=torch.float64, device="cuda:0")
    s.reset_accumulation()
    s.accumulate(cam, 0, 4096, depth, 1)
    s.resolve(out, acc)
    ref = acc / 4096

    def run(frames):
        s.reset_accumulation()
        rm = {}
        for k in range(frames):
            s.accumulate(cam, k, 1, depth, 0)
            if k + 1 in (4, 16, 64):
                s.resolve(out)
                rm[k + 1] = round(torch.sqrt(torch.mean((out.double() - ref) ** 2)).item(), 5)
        return rm

    s.reset_stats()
    plain = run(64)
    st = s.stats()
    rays_plain = st["extension_rays"] + st["shadow_rays"]
    s.set_radiance_cache(P.cache_config(train_paths=512, batch_size=4096))
    s.reset_stats()
    cached = run(64)
    st = s.stats()
    rays_cache = st["extension_rays"] + st["shadow_rays"]
    s.resolve(out)
    bias = float((out.double().mean() - ref.mean()) / ref.mean())
    # efficiency = 1 / (RMSE^2 x rays traced); rays include the training paths'
    gain = (plain[64] ** 2 * rays_plain) / (cached[64] ** 2 * rays_cache)
    _say(f"[nrc gain] RMSE plain {plain}  cache {cached}  mean bias of the cached image {bias:+.3%}; "
         f"rays plain {rays_plain}, cache {rays_cache} (incl. training paths), queries {st['cache_queries']}; "
         f"efficiency gain {gain:.3f}")
    assert cached[64] < plain[64]
    assert gain > 1.15
    assert abs(bias) < 0.05
    s.close()
