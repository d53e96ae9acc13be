"""Pins of four oracle routines that every other cache and anisotropy check
rests on (CPU only):

* the shading frame (tangent from the instance's object +z axis, the
  Duff et al. 2017 basis as its fallback) — closed forms, orthonormality,
  handedness, and the orientation of an anisotropic GGX lobe sampled
  through it (the brushed-metal anisotropy of the CAD-like scene, Sec. 4);
* the radiance cache's 12 inputs (Sec. 6.1 cache reading) — closed-form
  values of the spherical direction pairs, the box-normalised position, the
  albedos and the specular reflectance at normal incidence;
* Adam (Kingma & Ba 2015) at steps t >= 2 — constant, alternating and
  impulse gradients, whose bias-corrected moments have closed forms from
  geometric sums, pinning beta1, beta2 and the bias-correction exponent;
* bfloat16 rounding of the cache's tensor operands — against torch's own
  float32 -> bfloat16 conversion and against the definition (nearest
  bfloat16 value, ties to an even last mantissa bit) evaluated exactly in
  float64, on 10^6 values including exact ties, subnormals and overflow.
"""
import math

import numpy as np
import pytest

from oracle import nrc_np as N
from paper_2407_19977_amd import scenes


# ------------------------------------------------------------ shading frame --

def _rot(seed):
    """A uniformly random rotation (QR of a Gaussian matrix, det +1)."""
    r = np.random.Generator(np.random.PCG64(seed))
    q, rr = np.linalg.qr(r.normal(size=(3, 3)))
    q = q * np.sign(np.diag(rr))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _o2w(R, T=(0.0, 0.0, 0.0)):
    m = np.zeros((3, 4))
    m[:, :3] = R
    m[:, 3] = T
    return m.astype(np.float32)


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def test_frame_world_space_tangent_is_projected_z(O):
    r = np.random.Generator(np.random.PCG64(11))
    for _ in range(200):
        n = _unit(r.normal(size=3))
        if abs(n[2]) > 0.999:
            continue
        t, b = O.shading_frame(n)
        # the world +z axis with its normal component removed, normalised
        exp_t = _unit(np.array([0.0, 0.0, 1.0]) - n * n[2])
        assert np.allclose(t, exp_t, atol=1e-12)
        F = np.stack([t, b, n])
        assert np.allclose(F @ F.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(F) - 1.0) < 1e-12        # right-handed: t x b = n
        assert np.allclose(np.cross(t, b), n, atol=1e-12)


def test_frame_instance_tangent_follows_object_z(O):
    for seed in range(20):
        R = _rot(seed)
        Rf = _o2w(R, (1.0, -2.0, 3.0))
        Rd = Rf[:, :3].astype(np.float64)  # the oracle reads the float32 transform
        r = np.random.Generator(np.random.PCG64(100 + seed))
        n = _unit(r.normal(size=3))
        z = Rd[:, 2]                        # the object +z axis in world space
        p = z - n * np.dot(n, z)
        if np.linalg.norm(p) < 1e-2:
            continue
        t, b = O.shading_frame(n, Rf)
        assert np.allclose(t, _unit(p), atol=1e-12)
        assert np.allclose(b, np.cross(n, t), atol=1e-12)
        # translation does not matter
        t2, b2 = O.shading_frame(n, _o2w(R))
        assert np.array_equal(t, t2) and np.array_equal(b, b2)


def test_frame_fallback_closed_forms(O):
    # n parallel to the tangent axis: the projection vanishes and the
    # Duff et al. 2017 basis takes over; at the poles it is (x, +-y).
    t, b = O.shading_frame([0.0, 0.0, 1.0])
    assert np.allclose(t, [1, 0, 0], atol=0) and np.allclose(b, [0, 1, 0], atol=0)
    t, b = O.shading_frame([0.0, 0.0, -1.0])
    assert np.allclose(t, [1, 0, 0], atol=0) and np.allclose(b, [0, -1, 0], atol=0)
    # just inside the fallback radius (|projection| < 1e-3) the basis stays
    # orthonormal, right-handed and continuous with the pole's
    for eps in (1e-6, 1e-4, 8e-4):   # |projection| = 1.118 eps
        for sgn in (1.0, -1.0):
            n = _unit([eps, -0.5 * eps, sgn])
            t, b = O.shading_frame(n)
            F = np.stack([t, b, n])
            assert np.allclose(F @ F.T, np.eye(3), atol=1e-12)
            assert abs(np.linalg.det(F) - 1.0) < 1e-12
            assert np.linalg.norm(t - [1, 0, 0]) < 4 * eps
    # just outside it the projected axis is used again
    n = _unit([2e-3, 0.0, 1.0])
    t, _ = O.shading_frame(n)
    assert np.allclose(t, _unit(np.array([0.0, 0, 1]) - n * n[2]), atol=1e-12)
    # an instance whose object +z is the world x axis, seen along x
    R = np.array([[0.0, 0, 1], [0, 1, 0], [-1, 0, 0]])
    t, b = O.shading_frame([1.0, 0.0, 0.0], _o2w(R))
    F = np.stack([t, b, [1.0, 0, 0]])
    assert np.allclose(F @ F.T, np.eye(3), atol=1e-12) and abs(np.linalg.det(F) - 1) < 1e-12


def test_anisotropic_lobe_is_long_along_the_tangent(O):
    """Brushed metal (anisotropy 0.7): reflected directions sampled in the
    local frame and carried to world space through the oracle's frame spread
    most along the instance's projected +z axis, as the OpenPBR mapping
    alpha_t > alpha_b prescribes."""
    mat = scenes.material(base_metalness=1.0, base_color=(0.9, 0.9, 0.9), specular_roughness=0.3,
                          specular_roughness_anisotropy=0.7)
    a = 0.3 ** 2
    at = a * math.sqrt(2.0 / (1.0 + 0.3 ** 2))
    ab = 0.3 * at
    R = _rot(7)
    n = _unit([0.3, 0.9, -0.2])
    t, b = O.shading_frame(n, _o2w(R))
    z = R[:, 2]
    exp_t = _unit(z - n * np.dot(n, z))
    exp_b = np.cross(n, exp_t)
    r = np.random.Generator(np.random.PCG64(3))
    wo_l = np.array([0.0, 0.0, 1.0])
    along_t, along_b = [], []
    for _ in range(4000):
        s = O.bsdf_sample(mat, wo_l, r.uniform(0, 1, 4))
        if not s["ok"]:
            continue
        wl = s["wi"]
        ww = wl[0] * t + wl[1] * b + wl[2] * n      # local -> world through the frame
        along_t.append(np.dot(ww, exp_t))
        along_b.append(np.dot(ww, exp_b))
    st, sb = np.std(along_t), np.std(along_b)
    # at normal incidence the half vector spreads like alpha, the reflection twice as far
    assert st / sb == pytest.approx(at / ab, rel=0.15)
    assert st > 2.5 * sb


# ----------------------------------------------------------- cache inputs --

@pytest.mark.parametrize("wo,expect", [
    ((0.0, 0.0, -1.0), (0.5, 0.5)),      # horizon, phi = 0
    ((1.0, 0.0, 0.0), (0.5, 0.75)),      # horizon, phi = +pi/2
    ((-1.0, 0.0, 0.0), (0.5, 0.25)),     # horizon, phi = -pi/2
    ((0.0, -1.0, 0.0), (1.0, None)),     # straight down: theta = pi
    ((0.0, 1.0, 0.0), (0.0, None)),      # straight up: theta = 0
    ((0.5, math.sqrt(0.5), -0.5), (0.25, 0.625)),   # theta = pi/4, phi = pi/4
])
def test_cache_direction_pairs(O, wo, expect):
    lam = scenes.lambert((0.5, 0.5, 0.5))
    n = (0.0, 1.0, 0.0)
    x = O.nrc_inputs((0, 0, 0), (1, 1, 1), (0.5, 0.5, 0.5), wo, n, lam)
    assert x[3] == pytest.approx(expect[0], abs=1e-15)
    if expect[1] is not None:
        assert x[4] == pytest.approx(expect[1], abs=1e-15)
    # the normal's pair sits in its own slots: n = +y -> theta 0
    assert x[5] == 0.0
    # swapping the roles of wo and n swaps the slot pairs
    y = O.nrc_inputs((0, 0, 0), (1, 1, 1), (0.5, 0.5, 0.5), n, wo, lam)
    assert np.array_equal(y[3:5], x[5:7]) and np.array_equal(y[5:7], x[3:5])


def test_cache_position_albedo_and_specular_inputs(O):
    lo, hi = (-2.0, 0.0, 10.0), (2.0, 8.0, 14.0)
    wo, n = (0.0, 0.0, -1.0), (1.0, 0.0, 0.0)
    lam = scenes.material(base_weight=0.8, base_color=(0.5, 0.25, 1.0), specular_roughness=0.4,
                          specular_ior=1.5)
    x = O.nrc_inputs(lo, hi, (-2.0, 8.0, 11.0), wo, n, lam)
    assert np.allclose(x[0:3], [0.0, 1.0, 0.25], atol=1e-15)
    assert x[7] == pytest.approx(0.4, abs=1e-7)                 # roughness as given (float32)
    assert np.allclose(x[8:11], [0.4, 0.2, 0.8], atol=1e-7)       # base_weight * base_color
    assert x[11] == pytest.approx(((1.5 - 1) / (1.5 + 1)) ** 2, abs=1e-7)  # F(1, 1.5) = 0.04
    # a metal: no diffuse albedo, specular = luminance of base_weight * base_color
    metal = scenes.material(base_metalness=1.0, base_color=(1.0, 0.5, 0.0), specular_ior=1.5)
    x = O.nrc_inputs(lo, hi, (0.0, 4.0, 12.0), wo, n, metal)
    assert np.allclose(x[0:3], [0.5, 0.5, 0.5], atol=1e-15)
    assert np.all(x[8:11] == 0.0)
    assert x[11] == pytest.approx(0.2126 + 0.7152 * 0.5, abs=1e-7)
    # glass: transmission removes the diffuse albedo; the interface reflects F(1, 2) = 1/9 and
    # transmits the rest, so the specular albedo is 1
    glass = scenes.material(transmission_weight=1.0, specular_ior=2.0)
    x = O.nrc_inputs(lo, hi, (0.0, 4.0, 12.0), wo, n, glass)
    assert np.all(x[8:11] == 0.0)
    assert x[11] == pytest.approx(1.0, abs=1e-7)
    # half transmissive: 1/9 + 0.5 (8/9)
    half = scenes.material(transmission_weight=0.5, specular_ior=2.0, base_color=(0.2, 0.4, 0.6))
    x = O.nrc_inputs(lo, hi, (0.0, 4.0, 12.0), wo, n, half)
    assert np.allclose(x[8:11], [0.1, 0.2, 0.3], atol=1e-7)   # (1 - transmission 0.5) base_color
    assert x[11] == pytest.approx(1.0 / 9.0 + 0.5 * 8.0 / 9.0, abs=1e-7)
    # normal pair of n = +x: theta = pi/2, phi = pi/2
    assert np.allclose(x[5:7], [0.5, 0.75], atol=1e-15)


# ------------------------------------------------------------------ Adam --

B1, B2, LR, EPS = 0.9, 0.99, 1e-3, 1e-8


def _run_adam(gs):
    w = np.zeros(1)
    m = np.zeros(1)
    v = np.zeros(1)
    steps = []
    for t, g in enumerate(gs, start=1):
        w2, m, v = N.adam(w, m, v, np.array([g]), t)
        steps.append(float(w2[0] - w[0]))
        w = w2
    return steps


def test_adam_constant_gradient_steps_are_lr():
    # m_t = g (1 - b1^t), v_t = g^2 (1 - b2^t): the bias corrections undo
    # exactly the geometric sums, so every step is -lr g / (|g| + eps)
    for g in (3.0, -0.25):
        steps = _run_adam([g] * 6)
        for s in steps:
            assert s == pytest.approx(-LR * g / (abs(g) + EPS), rel=1e-12)


def test_adam_alternating_gradient_closed_form():
    # g_k = g (-1)^(k+1): m_t = (1-b1) g (-1)^(t+1) (1 - (-b1)^t) / (1 + b1),
    # v_t = (1-b2) g^2 (1 - b2^t) / (1 - b2) ... i.e. v_hat = g^2
    g = 2.0
    steps = _run_adam([g * (-1) ** k for k in range(8)])
    for t, s in enumerate(steps, start=1):
        mh = (1 - B1) * g * (-1) ** (t + 1) * (1 - (-B1) ** t) / ((1 + B1) * (1 - B1 ** t))
        assert s == pytest.approx(-LR * mh / (abs(g) + EPS), rel=1e-12)
    assert steps[1] == pytest.approx(LR / 19.0, rel=1e-6)   # t = 2: m_hat = -g (1-b1)/(1+b1) = -g/19


def test_adam_impulse_gradient_closed_form():
    # g at step 1, zero after: m_t = (1-b1) b1^(t-1) g, v_t = (1-b2) b2^(t-1) g^2
    g = -0.5
    steps = _run_adam([g] + [0.0] * 9)
    for t, s in enumerate(steps, start=1):
        mh = (1 - B1) * B1 ** (t - 1) * g / (1 - B1 ** t)
        vh = (1 - B2) * B2 ** (t - 1) * g * g / (1 - B2 ** t)
        assert s == pytest.approx(-LR * mh / (math.sqrt(vh) + EPS), rel=1e-12)
    # t = 2 in numbers: (b1/(1+b1)) / sqrt(b2/(1+b2)) lr
    assert abs(steps[1]) == pytest.approx(LR * (0.9 / 1.9) / math.sqrt(0.99 / 1.99), rel=1e-6)  # eps: 3e-8
    # a beta2 of 0.999 would move this step by 0.2 %
    assert abs(abs(steps[1]) - LR * (0.9 / 1.9) / math.sqrt(0.999 / 1.999)) > 1e-3 * abs(steps[1])


# --------------------------------------------- moving average of weights --

def _run_ema(ws, alpha):
    e = np.zeros(1)
    out = []
    for t, w in enumerate(ws, start=1):
        e = N.ema_update(e, np.array([w]), alpha)
        out.append(float(N.ema_weights(e, t, alpha, np.array([w]))[0]))
    return out


def test_ema_of_constant_weights_is_the_weights():
    # e_t = (1 - a^t) w: the bias correction returns w exactly at every step
    for a in (0.5, 0.9, 0.99):
        for v in _run_ema([1.75] * 12, a):
            assert v == pytest.approx(1.75, rel=1e-13)


def test_ema_of_linear_drift_closed_form():
    # w_t = t d: e_t / d = t (1 - a^t) - a (1 - t a^(t-1) + (t-1) a^t) / (1 - a)
    d = 0.3
    for a in (0.5, 0.9, 0.99):
        got = _run_ema([d * t for t in range(1, 11)], a)
        for t, v in enumerate(got, start=1):
            e = d * (t * (1 - a ** t) - a * (1 - t * a ** (t - 1) + (t - 1) * a ** t) / (1 - a))
            assert v == pytest.approx(e / (1 - a ** t), rel=1e-12)
    # the average lags the drift: at t = 2 with a = 0.9 it is (2 - a - a^2) d / (1 - a^2) = 1.4737 d
    assert _run_ema([d, 2 * d], 0.9)[1] == pytest.approx(d * (2 - 0.9 - 0.81) / (1 - 0.81), rel=1e-12)


def test_ema_off_and_before_the_first_step_is_the_weights():
    assert _run_ema([0.1, -4.0, 2.5], 0.0) == [0.1, -4.0, 2.5]
    w = np.array([0.25, -1.0])
    assert np.array_equal(N.ema_weights(np.zeros(2), 0, 0.99, w), w)


# -------------------------------------------------------------- bfloat16 --

def _bf16_by_definition(f32):
    """Nearest bfloat16 of each float32, ties to even, evaluated exactly in
    float64 from the two bfloat16 neighbours (no bit-add trick)."""
    u = f32.view(np.uint32).astype(np.int64)
    sign = u & 0x80000000
    mag = u & 0x7FFFFFFF
    lo = mag & 0x7FFF0000
    hi = lo + 0x10000
    x = np.abs(f32.astype(np.float64))
    lo_v = (lo.astype(np.uint32)).view(np.float32).astype(np.float64)
    hi_v = np.where(hi >= 0x7F800000, 2.0 ** 128,
                    (np.minimum(hi, 0x7F7F0000).astype(np.uint32)).view(np.float32).astype(np.float64))
    dlo, dhi = x - lo_v, hi_v - x
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((lo >> 16) & 1 == 1))
    r = np.where(pick_hi, hi, lo)
    r = np.where(pick_hi & (hi >= 0x7F800000), 0x7F800000, r)
    out = (r | sign).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def _bf16_test_values():
    r = np.random.Generator(np.random.PCG64(21))
    n = 10 ** 6
    bits = r.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    # replace inf/nan patterns by finite ones
    bits = np.where((bits & 0x7F800000) == 0x7F800000, bits & 0xBFFFFFFF, bits)
    k = n // 8
    # exact ties (low half 0x8000) with both parities of the kept bit
    bits[:k] = (bits[:k] & 0xFFFF0000) | 0x8000
    # subnormals and the smallest normals
    bits[k:2 * k] = (bits[k:2 * k] & 0x807FFFFF) | (r.integers(0, 2, k).astype(np.uint32) << 23)
    # values near the largest float32 (overflow to inf when rounding up)
    bits[2 * k:2 * k + 1000] = (bits[2 * k:2 * k + 1000] & 0x8000FFFF) | 0x7F7F0000
    # the cache's value range
    bits[3 * k:4 * k] = r.uniform(-4, 4, k).astype(np.float32).view(np.uint32)
    return bits.view(np.float32)


def test_bf16_numpy_equals_torch_and_definition():
    torch = pytest.importorskip("torch")
    f = _bf16_test_values()
    ref_t = torch.from_numpy(f.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    ref_d = _bf16_by_definition(f)
    ours = N.bf16(f)
    assert np.array_equal(ref_d, ref_t)           # the two references agree, infinities included
    assert np.array_equal(ours, ref_d)
    assert np.isinf(ref_d[2 * (10 ** 6 // 8):2 * (10 ** 6 // 8) + 1000]).any()


def test_bf16_c_oracle_equals_definition(O):
    f = _bf16_test_values()
    idx = np.concatenate([np.arange(0, 10 ** 6, 20), np.arange(2 * (10 ** 6 // 8), 2 * (10 ** 6 // 8) + 1000)])
    sub = f[idx]
    ref = _bf16_by_definition(sub)
    got = np.array([O.bf16_round(float(v)) for v in sub])
    assert np.array_equal(got, ref)
    # infinities and NaN pass through
    assert O.bf16_round(math.inf) == math.inf and math.isnan(O.bf16_round(math.nan))
