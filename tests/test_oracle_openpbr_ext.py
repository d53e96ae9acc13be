"""Pins of the oracle's OpenPBR additions (CPU only): the energy-preserving
Oren-Nayar diffuse (EON, Portsmouth, Kutz and Hill 2024, over Fujii's FON)
for base_diffuse_roughness, and the modulation of the dielectric IOR by
specular_weight (OpenPBR).

EON is pinned by what the model is built to satisfy and by closed forms:
white (albedo 1) EON reflects everything at every roughness and angle
(quadrature of f cos over the hemisphere); zero roughness is Lambert; the
value is reciprocal; the FON albedo E(mu) that the energy term uses equals
a quadrature of FON's own definition; the albedo of a grey EON is
rho E + rho_ms (1 - E).  The IOR modulation is pinned by the normal-incidence
reflectance xi F0(eta), by specular_weight 1 leaving the IOR alone, and by
smooth modulated glass staying lossless.
"""
import math

import numpy as np
import pytest

from paper_2407_19977_amd import scenes

M = scenes.material


def sph(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])


def _albedo_quad(O, mat, theta_o, n_t=160, n_p=192):
    """int f(wo, wi) cos(theta_i) dwi by Gauss-Legendre in cos(theta_i) and midpoints in phi."""
    wo = sph(theta_o, 0.4)
    x, w = np.polynomial.legendre.leggauss(n_t)
    mu = 0.5 * (x + 1.0)
    w = 0.5 * w
    tot = np.zeros(3)
    for m, wm in zip(mu, w):
        s = math.sqrt(max(0.0, 1.0 - m * m))
        acc = np.zeros(3)
        for k in range(n_p):
            p = (k + 0.5) * 2 * math.pi / n_p
            f, _ = O.bsdf_eval(mat, wo, np.array([s * math.cos(p), s * math.sin(p), m]))
            acc += f
        tot += wm * m * acc * (2 * math.pi / n_p)
    return tot


def _fon_AB(sigma):
    A = 1.0 / (1.0 + (0.5 - 2.0 / (3.0 * math.pi)) * sigma)
    return A, sigma * A


def _fon_albedo_quad(sigma, mu_o, n_t=200, n_p=256):
    """Albedo of FON with rho = 1 from its definition (A + B s/t)/pi, by quadrature."""
    A, B = _fon_AB(sigma)
    so = math.sqrt(1.0 - mu_o * mu_o)
    x, w = np.polynomial.legendre.leggauss(n_t)
    mu = 0.5 * (x + 1.0)
    w = 0.5 * w
    phis = (np.arange(n_p) + 0.5) * 2 * math.pi / n_p
    tot = 0.0
    for m, wm in zip(mu, w):
        si = math.sqrt(max(0.0, 1.0 - m * m))
        s = si * so * np.cos(phis)
        t = np.where(s > 0, max(m, mu_o), 1.0)
        tot += wm * m * np.sum((A + B * s / t) / math.pi) * (2 * math.pi / n_p)
    return tot


@pytest.mark.parametrize("sigma", [0.2, 0.6, 1.0])
@pytest.mark.parametrize("theta_o", [0.15, 0.9, 1.35, 1.55])
def test_white_eon_reflects_everything(O, sigma, theta_o):
    mat = M(base_color=(1.0, 1.0, 1.0), base_diffuse_roughness=sigma, specular_weight=0.0)
    a = _albedo_quad(O, mat, theta_o)
    assert np.allclose(a, 1.0, atol=2e-5), a


def test_grey_eon_albedo_closed_form(O):
    """rho E(mu_o) + rho_ms (1 - E(mu_o)), E from the quadrature of FON's definition."""
    for sigma, rho, th in ((0.5, 0.5, 0.7), (1.0, 0.3, 1.2), (0.8, 0.9, 0.3)):
        E = _fon_albedo_quad(sigma, math.cos(th))
        A, B = _fon_AB(sigma)
        Eb = A + B * (2.0 / 3.0 - 28.0 / (15.0 * math.pi))
        rho_ms = rho * rho * Eb / (1.0 - rho * (1.0 - Eb))
        expect = rho * E + rho_ms * (1.0 - E)
        a = _albedo_quad(O, M(base_color=(rho, rho, rho), base_diffuse_roughness=sigma, specular_weight=0.0), th)
        assert np.allclose(a, expect, atol=2e-5), (a, expect)
        # the FON albedo falls with roughness at normal incidence and is 1 for sigma = 0
    assert _fon_albedo_quad(0.0, 0.5) == pytest.approx(1.0, abs=1e-10)


def test_eon_mean_albedo_closed_form():
    """Eb = A + B (2/3 - 28/(15 pi)) is the cosine-weighted mean of E(mu) (quadrature of FON)."""
    x, w = np.polynomial.legendre.leggauss(24)
    mu = 0.5 * (x + 1.0)
    w = 0.5 * w
    for sigma in (0.3, 1.0):
        A, B = _fon_AB(sigma)
        Eb = sum(wi * 2 * m * _fon_albedo_quad(sigma, m, n_t=120, n_p=192) for m, wi in zip(mu, w))
        # nested midpoint / Gauss quadrature over the kinks of s/t is good to a few 1e-6
        assert Eb == pytest.approx(A + B * (2.0 / 3.0 - 28.0 / (15.0 * math.pi)), abs=1e-5)


def test_eon_zero_roughness_is_lambert_and_reciprocal(O):
    r = np.random.Generator(np.random.PCG64(5))
    lam = M(base_color=(0.6, 0.3, 0.2), specular_weight=0.0)
    for sigma in (0.0, 0.4, 1.0):
        mat = M(base_color=(0.6, 0.3, 0.2), base_diffuse_roughness=sigma, specular_weight=0.0)
        for _ in range(200):
            a, b = r.normal(size=3), r.normal(size=3)
            a[2], b[2] = abs(a[2]) + 1e-3, abs(b[2]) + 1e-3
            a /= np.linalg.norm(a)
            b /= np.linalg.norm(b)
            f1, _ = O.bsdf_eval(mat, a, b)
            f2, _ = O.bsdf_eval(mat, b, a)
            assert np.allclose(f1, f2, rtol=1e-12)
            if sigma == 0.0:
                assert np.array_equal(f1, O.bsdf_eval(lam, a, b)[0])
                assert np.allclose(f1, np.array([0.6, 0.3, 0.2]) / math.pi, rtol=1e-7)
    # retro-reflection: with wi = wo the FON term has s = sin^2(theta) > 0 and t = cos(theta), so rough
    # diffuse grows toward grazing retro-reflection while Lambert stays flat
    rough = M(base_color=(1, 1, 1), base_diffuse_roughness=1.0, specular_weight=0.0)
    f_n = O.bsdf_eval(rough, sph(0.0, 0.0), sph(0.0, 0.0))[0][0]
    f_g = O.bsdf_eval(rough, sph(1.3, 0.0), sph(1.3, 0.0))[0][0]
    assert f_g > 1.5 * f_n


def test_specular_weight_modulates_the_ior(O):
    """F(1, eta') = xi F0(eta): the cache's specular input of a dielectric is that reflectance."""
    for eta in (1.5, 1.33, 2.4, 0.8):
        F0 = ((eta - 1.0) / (eta + 1.0)) ** 2
        for xi in (0.0, 0.3, 0.6, 1.0):
            mat = M(base_color=(0.5, 0.5, 0.5), specular_weight=xi, specular_ior=eta)
            x = O.nrc_inputs((0, 0, 0), (1, 1, 1), (0.5, 0.5, 0.5), (0, 0, 1), (0, 0, 1), mat)
            e32 = float(np.float32(eta))
            F0_32 = ((e32 - 1.0) / (e32 + 1.0)) ** 2
            assert x[11] == pytest.approx(float(np.float32(xi)) * F0_32, rel=1e-12, abs=1e-15), (eta, xi)
    # smooth glass with a weak specular: reflection + refraction still carry everything
    glass = M(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.0, specular_ior=1.5,
              specular_weight=0.5)
    wo = sph(0.8, 0.2)
    r = math.sqrt(0.5 * 0.04)
    eta_mod = (1.0 + r) / (1.0 - r)   # 1.3294: the refraction bends by the modulated IOR
    tot = np.zeros(3)
    for u in np.linspace(0.0005, 0.9995, 400):
        s = O.bsdf_sample(glass, wo, [0.5, 0.3, 0.6, u])
        w = s["weight"] * (eta_mod ** 2 if s["refract"] else 1.0)   # radiance scaling 1/eta'^2 undone
        tot += w / 400
    assert np.allclose(tot, 1.0, atol=1e-9), tot
