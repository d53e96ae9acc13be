"""Pins of the oracle's fuzz lobe (CPU only).

OpenPBR (named by the paper, Sec. 4) puts an optional fuzz layer on top of
the material.  The oracle's reading: a sheen lobe with the "Charlie"
distribution D(h) = (2 + 1/a) sin^(1/a)(theta_h) / (2 pi) and the visibility
1 / (4 (mu_i + mu_o - mu_i mu_o)), over layers attenuated by
(1 - w E(mu_i)) (1 - w E(mu_o)), E the lobe's directional albedo from a
table.  Pinned by what does not depend on the code that computes it: the
distribution's projected area integrates to one; the table equals the
albedo integrated from the evaluated lobe, and its closed form at normal
incidence for a = 1; the white furnace of fuzz over a white Lambert base
follows the layering's closed form and stays below one; reciprocity; a
fuzz weight of zero leaves the base; and the fuzz material passes the BSDF
consistency, energy and chi-square checks of test_oracle_bsdf.py.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2407_19977_amd import scenes

M = scenes.material


def _fuzz_only(rough, w=1.0, color=(1.0, 1.0, 1.0)):
    # no base, no specular: only the fuzz lobe reflects
    return M(base_weight=0.0, specular_weight=0.0, fuzz_weight=w, fuzz_color=color, fuzz_roughness=rough)


def _sph(t, p):
    return np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])


def _hemi_quad(fn, nt=96, npf=96):
    """Gauss-Legendre in cos(theta) times the midpoint rule in phi over the upper hemisphere."""
    x, w = np.polynomial.legendre.leggauss(nt)
    mus = 0.5 * (x + 1.0)
    ws = 0.5 * w
    tot = 0.0
    for mu, wt in zip(mus, ws):
        s = math.sqrt(max(0.0, 1.0 - mu * mu))
        acc = 0.0
        for k in range(npf):
            p = 2 * math.pi * (k + 0.5) / npf
            acc += fn(np.array([s * math.cos(p), s * math.sin(p), mu]))
        tot += wt * acc * 2 * math.pi / npf
    return tot


@pytest.mark.parametrize("rough", [0.3, 0.6, 1.0])
def test_distribution_is_normalised(O, rough):
    """Recover D(theta_h) from the evaluated lobe at wo = wi = h (the mirror configuration of h
    itself: D = f 4 (mu_i + mu_o - mu_i mu_o) there) and integrate D cos(theta_h) over half
    vectors: the projected microfacet area is one."""
    mat = _fuzz_only(rough)
    def D(th):
        h = np.array([math.sin(th), 0.0, math.cos(th)])
        f, _ = O.bsdf_eval(mat, h, h)
        mu = h[2]
        return f[0] * 4.0 * (2.0 * mu - mu * mu)
    total = integrate.quad(lambda th: D(th) * math.cos(th) * math.sin(th) * 2 * math.pi, 0.0,
                           math.pi / 2 - 1e-9, limit=400, epsabs=1e-12)[0]
    assert total == pytest.approx(1.0, abs=2e-6)


@pytest.mark.parametrize("rough", [0.2, 0.5, 0.9])
def test_albedo_table_matches_the_integrated_lobe(O, rough):
    mat = _fuzz_only(rough)
    for th in (0.0, 0.5, 1.0, 1.3):
        wo = _sph(th, 0.0)
        est = _hemi_quad(lambda wi: O.bsdf_eval(mat, wo, wi)[0][0] * wi[2])
        assert O.fuzz_albedo(rough, wo[2]) == pytest.approx(est, rel=2e-3, abs=2e-4)


def test_albedo_at_normal_incidence_closed_form(O):
    # a = 1 (roughness 1): D = 3 sin(theta_h) / (2 pi); at wo = n, theta_h = theta_i / 2 and V = 1/4
    want = integrate.quad(lambda t: 0.75 * math.sin(t / 2) * math.cos(t) * math.sin(t), 0.0, math.pi / 2,
                          epsabs=1e-13)[0]
    assert O.fuzz_albedo(1.0, 1.0) == pytest.approx(want, rel=1e-4)


@pytest.mark.parametrize("rough", [0.3, 0.8])
def test_white_furnace_of_fuzz_over_white_lambert(O, rough):
    """Total albedo = E(mu_o) + (1 - E(mu_o)) (1 - Ebar) with Ebar = 2 int E(mu) mu dmu,
    the closed form of the layering over an albedo-1 Lambert base; it stays below one."""
    mat = M(base_color=(1.0, 1.0, 1.0), specular_weight=0.0, fuzz_weight=1.0, fuzz_roughness=rough)
    x, w = np.polynomial.legendre.leggauss(200)
    mus = 0.5 * (x + 1.0)
    Ebar = float(np.sum(0.5 * w * 2.0 * np.array([O.fuzz_albedo(rough, m) for m in mus]) * mus))
    for th in (0.1, 0.8, 1.2):
        wo = _sph(th, 0.3)
        E = O.fuzz_albedo(rough, wo[2])
        total = _hemi_quad(lambda wi: O.bsdf_eval(mat, wo, wi)[0][1] * wi[2], nt=128, npf=128)
        assert total == pytest.approx(E + (1.0 - E) * (1.0 - Ebar), rel=2e-3)
        assert total < 1.0


def test_reciprocity_and_zero_weight(O):
    mat = M(base_color=(0.4, 0.5, 0.6), specular_roughness=0.4, fuzz_weight=0.8, fuzz_color=(0.9, 0.6, 0.3),
            fuzz_roughness=0.4)
    base = M(base_color=(0.4, 0.5, 0.6), specular_roughness=0.4)
    none = M(base_color=(0.4, 0.5, 0.6), specular_roughness=0.4, fuzz_weight=0.0, fuzz_color=(0.9, 0.6, 0.3),
             fuzz_roughness=0.4)
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(200):
        a, b = rng.normal(size=3), rng.normal(size=3)
        a[2], b[2] = abs(a[2]) + 1e-3, abs(b[2]) + 1e-3
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        f1, _ = O.bsdf_eval(mat, a, b)
        f2, _ = O.bsdf_eval(mat, b, a)
        assert np.allclose(f1, f2, rtol=1e-12)
        g1, p1 = O.bsdf_eval(base, a, b)
        g2, p2 = O.bsdf_eval(none, a, b)
        assert np.array_equal(g1, g2) and p1 == p2
