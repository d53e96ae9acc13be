"""Pins of the display oracle (CPU only): the Khronos PBR Neutral tone
mapper, the sRGB transfer function and the 8-bit display image (Sec. 5.1.4:
the running mean is tone mapped with PBR Neutral and shown after every
sampling iteration).

PBR Neutral is pinned by closed forms of its branches: colours whose
smallest channel is at least 0.08 and whose peak stays below the start of
compression move down by exactly 0.04; a darker minimum x moves the colour
by x - 6.25 x^2 (so black stays black and the two branches meet at 0.08);
a grey g >= 0.8 maps to 1 - 0.0576 / (g - 0.56); the branches are
continuous at the start of compression; saturated highlights desaturate to
white.  sRGB is pinned by its end points, its continuity at the knee and
the inverse (decode) transfer function.
"""
import numpy as np
import pytest


def test_pbr_neutral_linear_branch(O):
    r = np.random.Generator(np.random.PCG64(1))
    for _ in range(200):
        c = r.uniform(0.08, 0.79, 3)
        if c.max() - 0.04 >= 0.76:
            continue
        assert np.allclose(O.pbr_neutral(c), c - 0.04, atol=1e-15)
    # dark minimum: offset x - 6.25 x^2
    for x in (0.0, 0.01, 0.05, 0.0799):
        c = np.array([x, 0.3, 0.5])
        off = x - 6.25 * x * x
        assert np.allclose(O.pbr_neutral(c), c - off, atol=1e-15)
    assert np.array_equal(O.pbr_neutral([0.0, 0.0, 0.0]), [0.0, 0.0, 0.0])
    # the two offsets meet at x = 0.08
    assert 0.08 - 6.25 * 0.08 ** 2 == pytest.approx(0.04, abs=1e-15)


def test_pbr_neutral_grey_compression_closed_form(O):
    for g in (0.8, 0.9, 1.0, 2.0, 10.0, 1e3):
        out = O.pbr_neutral([g, g, g])
        assert np.allclose(out, 1.0 - 0.0576 / (g - 0.56), rtol=0, atol=1e-14), g
    # continuity at the start of compression (peak 0.76 after the offset)
    below = O.pbr_neutral([0.8 - 1e-12] * 3)
    above = O.pbr_neutral([0.8 + 1e-12] * 3)
    assert np.allclose(below, 0.76, atol=1e-11) and np.allclose(above, 0.76, atol=1e-11)
    # monotone along the grey ramp, bounded by 1
    ramp = np.geomspace(1e-4, 1e5, 400)
    vals = np.array([O.pbr_neutral([v, v, v])[0] for v in ramp])
    assert np.all(np.diff(vals) > 0) and vals.max() < 1.0


def test_pbr_neutral_highlights_desaturate(O):
    prev = None
    for k in (1.0, 3.0, 10.0, 100.0, 1e4):
        out = O.pbr_neutral([k, 0.0, 0.0])
        assert np.all(out <= 1.0 + 1e-15) and np.all(out >= 0.0)
        sat = out[0] - out[1]
        if prev is not None:
            assert sat < prev       # brighter red is less saturated
        prev = sat
        assert out[1] == pytest.approx(out[2], abs=1e-15)
    assert np.allclose(O.pbr_neutral([1e8, 0.0, 0.0]), 1.0, atol=1e-6)
    # below compression, hue is kept exactly: the offset is the same for every channel
    c = np.array([0.7, 0.2, 0.1])
    o = O.pbr_neutral(c)
    assert np.allclose(c - o, (c - o)[0], atol=1e-15)


def _srgb_decode(e):
    """IEC 61966-2-1 decoding (the inverse transfer function)."""
    return e / 12.92 if e <= 0.04045 else ((e + 0.055) / 1.055) ** 2.4


def test_srgb_transfer(O):
    assert O.srgb_encode(0.0) == 0.0 and O.srgb_encode(1.0) == 1.0
    assert O.srgb_encode(-1.0) == 0.0 and O.srgb_encode(5.0) == 1.0
    knee = 0.0031308
    assert abs(O.srgb_encode(knee * (1 - 1e-12)) - O.srgb_encode(knee * (1 + 1e-12))) < 1e-7
    for v in np.geomspace(1e-6, 1.0, 300):
        assert _srgb_decode(O.srgb_encode(v)) == pytest.approx(v, rel=1e-5, abs=1e-9)
    # mid grey: linear 0.5 encodes to 0.7354 (188 of 255)
    assert O.srgb_encode(0.5) == pytest.approx(0.735356983, abs=1e-8)
    assert int(np.floor(255 * O.srgb_encode(0.5) + 0.5)) == 188


def test_display_image_composes_the_steps(O):
    r = np.random.Generator(np.random.PCG64(2))
    spp = 16
    mean = np.concatenate([r.uniform(0, 1.5, (20, 30, 3)), r.exponential(3.0, (20, 30, 3))], 0)
    mean[0, 0] = 0.0
    mean[0, 1] = [1e6, 1e6, 1e6]
    enc, rgba = O.display(mean * spp, spp, exposure=0.7)
    for (y, x) in [(0, 0), (0, 1), (3, 7), (25, 11), (39, 29)]:
        t = O.pbr_neutral(mean[y, x] * 0.7)
        e = np.array([O.srgb_encode(v) for v in t])
        assert np.allclose(enc[y, x], e, atol=1e-15)
        assert np.array_equal(rgba[y, x, :3], np.floor(255 * e + 0.5).astype(np.uint8))
    assert np.all(rgba[..., 3] == 255)
    assert np.array_equal(rgba[0, 0, :3], [0, 0, 0])
    assert np.all(rgba[0, 1, :3] == 255)
    assert enc.min() >= 0.0 and enc.max() <= 1.0
