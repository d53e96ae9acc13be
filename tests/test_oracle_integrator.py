"""Pins of the oracle's estimator (CPU only).

The estimator is the Monte Carlo integration of the rendering equation
(Sec. 1.1) with importance sampling and Russian roulette (Sec. 5.1.3) plus
next-event estimation with MIS.  Closed-form scenes pin it:

* white furnace: albedo-1 diffuse objects under a uniform sky of radiance 1
  return 1 (exactly per sample for a convex object with BSDF sampling only);
* a smooth glass sphere under a uniform sky returns 1 per escaping sample;
* a Lambert plane of albedo rho under an upper-hemisphere sky L gives rho*L;
* the MIS, BSDF-only and NEE-only estimators, and Russian roulette on/off,
  agree in expectation on the closed box scene;
* the error of the box scene falls as spp^-1/2.
"""
import math

import numpy as np
import pytest

from paper_2407_19977_amd import scenes


def test_furnace_convex_bsdf_only_is_exact(O):
    sc = scenes.furnace("sphere", width=16, height=16, spp=4, max_depth=5)
    os_ = O.OracleScene(sc)
    r = os_.render(4, 5, estimator=O.BSDF_ONLY, per_sample=True)
    assert np.allclose(r["per_sample"], 1.0, rtol=0, atol=1e-12)


def test_furnace_convex_mis_unbiased(O):
    sc = scenes.furnace("sphere", width=16, height=16, spp=64, max_depth=5)
    os_ = O.OracleScene(sc)
    r = os_.render(64, 5, per_sample=True)
    v = r["per_sample"].reshape(-1, 3)
    mean, se = v.mean(0), v.std(0) / math.sqrt(len(v))
    assert np.all(np.abs(mean - 1.0) < 4 * se + 1e-12)
    assert v.std() > 0  # MIS mixes two strategies, so samples are not all 1


def test_furnace_concave_with_roulette(O):
    sc = scenes.furnace("cubes", width=16, height=16, spp=32, max_depth=256)
    os_ = O.OracleScene(sc)
    r = os_.render(32, 256, per_sample=True)
    ps = r["per_sample"]
    v = ps.reshape(-1, 3)
    mean, se = v.mean(0), v.std(0) / math.sqrt(len(v))
    assert np.all(np.abs(mean - 1.0) < 4 * se)
    # every pixel within 5 sigma of 1
    pm = ps.mean(2)
    psd = ps.std(2) / math.sqrt(ps.shape[2]) + 1e-9
    assert np.all(np.abs(pm - 1.0) < 5 * psd + 1e-9)


def test_furnace_smooth_glass_sphere(O):
    sc = scenes.furnace("glass", width=24, height=24, spp=8, max_depth=64)
    os_ = O.OracleScene(sc)
    r = os_.render(8, 64, per_sample=True)
    v = r["per_sample"]
    one = np.isclose(v, 1.0, rtol=0, atol=1e-9).all(-1)
    zero = (v == 0).all(-1)
    assert np.all(one | zero)           # escaping samples carry exactly the sky radiance
    assert zero.mean() < 0.01           # truncation at depth 64 is rare


@pytest.mark.parametrize("estimator", ["bsdf", "mis", "nee"])
def test_diffuse_plane_under_sky(O, estimator):
    rho = (0.3, 0.5, 0.7)
    L = 2.0
    sc = scenes.plane(rho=rho, L=L, width=24, height=24)
    os_ = O.OracleScene(sc)
    est = {"bsdf": O.BSDF_ONLY, "mis": O.MIS, "nee": O.NEE_ONLY}[estimator]
    r = os_.render(16, 3, estimator=est, per_sample=True)
    ps = r["per_sample"]
    rho32 = np.array(rho, dtype=np.float32).astype(np.float64)
    expect_plane = rho32 * L
    # classify pixels by the primary hit of sample 0's ray through the pixel centre
    plane_px = []
    for y in range(sc.camera.height):
        for x in range(sc.camera.width):
            o, d = O.camera_ray(sc.camera, x + 0.5, y + 0.5)
            plane_px.append(d[1] < -0.05)
    plane_px = np.array(plane_px).reshape(sc.camera.height, sc.camera.width)
    sky_px = np.array([[O.camera_ray(sc.camera, x + 0.5, y + 0.5)[1][1] > 0.05 for x in range(sc.camera.width)]
                       for y in range(sc.camera.height)])
    assert plane_px.sum() > 100 and sky_px.sum() > 50
    assert np.allclose(ps[sky_px], L, atol=1e-12)
    v = ps[plane_px].reshape(-1, 3)
    if estimator == "bsdf":
        assert np.allclose(v, expect_plane, rtol=1e-12)
    else:
        mean, se = v.mean(0), v.std(0) / math.sqrt(len(v))
        assert np.all(np.abs(mean - expect_plane) < 4 * se + 1e-12)


def _block_z(a, b, na, nb, blk=16):
    """z-scores of block means of two independent per-sample renders [h,w,n,3]."""
    h, w = a.shape[:2]
    zs = []
    for y in range(0, h, blk):
        for x in range(0, w, blk):
            va = a[y:y + blk, x:x + blk].reshape(-1, 3).sum(1)
            vb = b[y:y + blk, x:x + blk].reshape(-1, 3).sum(1)
            se = math.sqrt(va.var() / len(va) + vb.var() / len(vb)) + 1e-12
            zs.append((va.mean() - vb.mean()) / se)
    return np.array(zs)


def test_estimators_agree_on_box(O):
    sc = scenes.cornell(width=64, height=64)
    os_ = O.OracleScene(sc)
    ref = os_.render(32, 4, seed=11, per_sample=True)["per_sample"]
    for est in (O.BSDF_ONLY, O.NEE_ONLY):
        other = os_.render(32, 4, seed=12, estimator=est, per_sample=True)["per_sample"]
        z = _block_z(ref, other, 32, 32)
        assert np.all(np.abs(z) < 4.5), (est, z)
    rr_off = os_.render(32, 4, seed=13, rr=False, per_sample=True)["per_sample"]
    z = _block_z(ref, rr_off, 32, 32)
    assert np.all(np.abs(z) < 4.5), z


def test_error_falls_as_inverse_sqrt_spp(O):
    sc = scenes.cornell(width=128, height=128)
    os_ = O.OracleScene(sc)
    crop = (48, 48, 32, 32)
    ref = os_.render(4096, 4, seed=99, crop=crop)["mean"]
    spps = [4, 16, 64, 256]
    rmse = [math.sqrt(np.mean((os_.render(s, 4, seed=1, crop=crop)["mean"] - ref) ** 2)) for s in spps]
    slope = np.polyfit(np.log(spps), np.log(rmse), 1)[0]
    assert -0.6 < slope < -0.4, (slope, rmse)


def test_signature_is_deterministic_and_path_specific(O):
    sc = scenes.cornell(width=32, height=32)
    os_ = O.OracleScene(sc)
    a = os_.render(4, 4, per_sample=True)
    b = os_.render(4, 4, per_sample=True)
    assert np.array_equal(a["sigs"], b["sigs"]) and np.array_equal(a["per_sample"], b["per_sample"])
    # paths that leave through the open front share one signature; the rest are mostly distinct
    assert len(np.unique(a["sigs"])) > 0.3 * a["sigs"].size
    rgb, sig = os_.trace_path(5, 7, 2, 4)
    assert sig == int(a["sigs"][7, 5, 2]) and np.array_equal(rgb, a["per_sample"][7, 5, 2])
