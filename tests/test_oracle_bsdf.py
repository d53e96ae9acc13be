"""Pins of the oracle's OpenPBR BSDF (CPU only).

The paper uses OpenPBR (Sec. 4) for metallic, glossy and diffuse surfaces
with importance sampling (Sec. 5.1.3) but prints no formulas; the model is
pinned here by what the mathematics fixes: Fresnel closed forms from Snell's
law, the F82-tint anchor points, normalisation of the GGX distribution and of
its visible-normal density, sampler/pdf consistency, Lambert's exact weight,
reciprocity, energy bounds and chi-square agreement of sampled directions
with the evaluated pdf.
"""
import math

import numpy as np
import pytest

from paper_2407_19977_amd import scenes

M = scenes.material
MATS = {
    "lambert_white": scenes.lambert((1.0, 1.0, 1.0)),
    "lambert": scenes.lambert((0.7, 0.4, 0.2)),
    "metal": M(base_color=(0.9, 0.6, 0.3), base_metalness=1.0, specular_roughness=0.4),
    "metal_aniso": M(base_color=(0.8, 0.8, 0.9), base_metalness=1.0, specular_roughness=0.5,
                     specular_roughness_anisotropy=0.7, specular_color=(0.9, 0.7, 0.8)),
    "plastic": M(base_color=(0.5, 0.3, 0.2), specular_roughness=0.5, specular_ior=1.5),
    "coated_delta": M(base_color=(0.5, 0.3, 0.2), specular_roughness=0.3, specular_ior=1.5,
                      coat_weight=1.0, coat_ior=1.5, coat_roughness=0.0),
    "coated_rough": M(base_color=(0.1, 0.6, 0.8), specular_roughness=0.4, coat_weight=0.8,
                      coat_ior=1.5, coat_roughness=0.2, coat_color=(0.9, 0.9, 0.7)),
    "half_metal": M(base_color=(0.6, 0.6, 0.6), base_metalness=0.5, specular_roughness=0.35),
    "glass_rough": M(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.3, specular_ior=1.5),
    "glass_tinted": M(base_weight=0.0, transmission_weight=0.7, transmission_color=(0.9, 0.5, 0.5),
                      specular_roughness=0.45, specular_ior=1.33, base_color=(0.3, 0.3, 0.3)),
    "eon": M(base_color=(0.7, 0.4, 0.2), base_diffuse_roughness=0.8, specular_weight=0.0),
    "eon_plastic_weak": M(base_color=(0.5, 0.3, 0.2), base_diffuse_roughness=0.4, specular_roughness=0.4,
                          specular_weight=0.5),
    "plastic_film": M(base_color=(0.5, 0.3, 0.2), specular_roughness=0.4, thin_film_weight=1.0,
                      thin_film_thickness=0.35, thin_film_ior=1.33),
    "glass_film": M(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.3, specular_ior=1.5,
                    thin_film_weight=0.8, thin_film_thickness=0.5, thin_film_ior=1.38),
    "fuzz_plastic": M(base_color=(0.5, 0.3, 0.2), specular_roughness=0.4, fuzz_weight=0.7,
                      fuzz_color=(0.9, 0.8, 0.6), fuzz_roughness=0.4),
    "fuzz_coated": M(base_color=(0.2, 0.3, 0.6), specular_roughness=0.3, coat_weight=1.0, coat_roughness=0.0,
                     fuzz_weight=0.5, fuzz_roughness=0.8),
    "subsurface_eon": M(base_color=(0.7, 0.3, 0.2), base_diffuse_roughness=0.5, specular_roughness=0.3,
                        subsurface_weight=0.6, subsurface_color=(0.9, 0.8, 0.6)),
}
OPAQUE = ["lambert", "metal", "metal_aniso", "plastic", "coated_delta", "coated_rough", "half_metal", "eon",
          "eon_plastic_weak", "plastic_film", "fuzz_plastic", "fuzz_coated", "subsurface_eon"]


def sph(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])


def rng_dirs(n, seed, upper=True):
    r = np.random.Generator(np.random.PCG64(seed))
    v = r.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    if upper:
        v[:, 2] = np.abs(v[:, 2])
    return v


# ------------------------------------------------------------- Fresnel --

def test_fresnel_closed_forms(O):
    assert abs(O.fresnel_dielectric(1.0, 1.5) - 0.04) < 1e-15
    assert abs(O.fresnel_dielectric(1.0, 1.33) - ((0.33 / 2.33) ** 2)) < 1e-15
    assert O.fresnel_dielectric(0.0, 1.5) == 1.0
    # total internal reflection beyond the critical angle asin(eta) for eta < 1
    eta = 1.0 / 1.5
    crit = math.asin(eta)
    for th in np.linspace(crit + 1e-6, math.pi / 2, 20):
        assert O.fresnel_dielectric(math.cos(th), eta) == 1.0
    # Brewster angle: tan(theta_B) = eta makes Rp = 0, so F = Rs / 2
    for eta in (1.5, 1.33, 2.4, 1.0 / 1.5):
        tb = math.atan(eta)
        ci = math.cos(tb)
        ct = math.sqrt(1 - (math.sin(tb) / eta) ** 2)
        rs = ((ci - eta * ct) / (ci + eta * ct)) ** 2
        assert abs(O.fresnel_dielectric(ci, eta) - rs / 2) < 1e-14


def test_fresnel_matches_snell_form(O):
    # textbook unpolarised reflectance from Snell's law, (Rs + Rp) / 2
    for eta in (1.5, 1.33, 1.0 / 1.5, 2.0):
        for th in np.linspace(0.0, math.pi / 2 - 1e-3, 57):
            ci = math.cos(th)
            s2 = (math.sin(th) / eta) ** 2
            if s2 >= 1.0:
                expect = 1.0
            else:
                ct = math.sqrt(1 - s2)
                rs = ((ci - eta * ct) / (ci + eta * ct)) ** 2
                rp = ((eta * ci - ct) / (eta * ci + ct)) ** 2
                expect = 0.5 * (rs + rp)
            assert abs(O.fresnel_dielectric(ci, eta) - expect) < 1e-13


def test_f82_anchor_points(O):
    m = M(base_color=(0.9, 0.5, 0.2), base_weight=0.8, base_metalness=1.0, specular_color=(0.7, 0.9, 1.0))
    F0 = 0.8 * np.array([0.9, 0.5, 0.2], dtype=np.float32).astype(np.float64)
    sc = np.array([0.7, 0.9, 1.0], dtype=np.float32).astype(np.float64)
    assert np.allclose(O.fresnel_f82(m, 1.0), F0, atol=1e-7)
    assert np.allclose(O.fresnel_f82(m, 0.0), 1.0, atol=1e-15)
    mb = 1.0 / 7.0
    S = F0 + (1 - F0) * (1 - mb) ** 5
    assert np.allclose(O.fresnel_f82(m, mb), sc * S, atol=1e-7)
    # a white tint reduces F82 to Schlick's approximation
    w = M(base_color=(0.9, 0.5, 0.2), base_metalness=1.0)
    for mu in np.linspace(0, 1, 11):
        F0w = np.array([0.9, 0.5, 0.2], dtype=np.float32).astype(np.float64)
        assert np.allclose(O.fresnel_f82(w, mu), F0w + (1 - F0w) * (1 - mu) ** 5, atol=1e-14)


# ------------------------------------------------------------------ GGX --

def _hemi_quad(f, amax, n_t=240, n_p=96):
    """Integrate f(m) over the upper hemisphere; theta = atan(amax * tan(pi/2 v)), Gauss-Legendre in v."""
    xv, wv = np.polynomial.legendre.leggauss(n_t)
    v = 0.5 * (xv + 1.0)
    wv = 0.5 * wv
    x = amax * np.tan(0.5 * np.pi * v)
    theta = np.arctan(x)
    dtheta_dv = amax * 0.5 * np.pi / np.cos(0.5 * np.pi * v) ** 2 / (1 + x * x)
    phis = (np.arange(n_p) + 0.5) * 2 * np.pi / n_p
    tot = 0.0
    for t, w, j in zip(theta, wv, dtheta_dv):
        s = 0.0
        for p in phis:
            s += f(sph(t, p))
        tot += w * j * math.sin(t) * s * (2 * np.pi / n_p)
    return tot


@pytest.mark.parametrize("at,ab", [(0.3, 0.3), (0.5, 0.1), (0.05, 0.05), (0.8, 0.8)])
def test_ggx_D_normalised(O, at, ab):
    # int D(m) (m.n) dm = 1
    val = _hemi_quad(lambda m: O.ggx_D(at, ab, m) * m[2], max(at, ab))
    assert abs(val - 1.0) < 2e-3


@pytest.mark.parametrize("at,ab,theta_o", [(0.3, 0.3, 0.4), (0.5, 0.1, 1.2), (0.2, 0.4, 1.5), (0.6, 0.6, 0.0)])
def test_ggx_weak_white_furnace(O, at, ab, theta_o):
    # int G1(wo) max(0, wo.m) D(m) / wo.z dm = 1  (Heitz 2014): the visible-normal density integrates to 1
    wo = sph(theta_o, 0.7)
    val = _hemi_quad(lambda m: O.ggx_vndf_pdf(at, ab, wo, m), max(at, ab))
    assert abs(val - 1.0) < 3e-3


@pytest.mark.parametrize("at,ab,theta_o", [(0.3, 0.3, 0.5), (0.6, 0.15, 1.3)])
def test_vndf_sampler_matches_density(O, at, ab, theta_o):
    # moments of sampled normals equal the moments of the density: E[phi(m)] = int phi pdf dm
    wo = sph(theta_o, 2.0)
    n = 20000
    ms = np.empty((n, 3))
    for i in range(n):
        u1, u2 = O.uniform(3, i, 0, 0, 4), O.uniform(3, i, 0, 0, 5)
        m = O.ggx_vndf_sample(at, ab, wo, u1, u2)
        assert O.ggx_vndf_pdf(at, ab, wo, m) > 0
        assert abs(np.linalg.norm(m) - 1) < 1e-12
        ms[i] = m
    phis = [lambda m: m[..., 2], lambda m: m[..., 0] ** 2, lambda m: (m[..., 1] > 0).astype(float),
            lambda m: m[..., 0] * m[..., 1]]
    for phi in phis:
        mc = phi(ms)
        q = _hemi_quad(lambda m: phi(m) * O.ggx_vndf_pdf(at, ab, wo, m), max(at, ab))
        assert abs(mc.mean() - q) < 4 * mc.std() / math.sqrt(n) + 2e-3


# ---------------------------------------------------------------- BSDF --

def _u(i, salt=0):
    return [np.random.Generator(np.random.PCG64(1000 * salt + i)).uniform(size=4)][0]


@pytest.mark.parametrize("name", list(MATS))
def test_sample_weight_and_pdf_consistent(O, name):
    mat = MATS[name]
    for i in range(400):
        wo = rng_dirs(1, 17 * i + 1)[0]
        if wo[2] < 1e-3:
            continue
        entering = 1 if i % 3 else 0
        s = O.bsdf_sample(mat, wo, _u(i, 1), entering=entering)
        if not s["ok"]:
            continue
        assert abs(np.linalg.norm(s["wi"]) - 1.0) < 1e-12
        if s["delta"]:
            continue
        f, pdf = O.bsdf_eval(mat, wo, s["wi"], entering=entering)
        assert s["pdf"] == pytest.approx(pdf, rel=1e-12)
        expect = f * abs(s["wi"][2]) / pdf
        assert np.allclose(s["weight"], expect, rtol=1e-12, atol=0)


def test_lambert_weight_is_albedo(O):
    mat = MATS["lambert"]
    rho = np.asarray(mat[1:4], dtype=np.float64)
    for i in range(300):
        wo = rng_dirs(1, i + 5)[0]
        s = O.bsdf_sample(mat, wo, _u(i, 2))
        assert s["ok"] and s["lobe"] == 4
        assert np.allclose(s["weight"], rho, rtol=1e-14)
        assert s["pdf"] == pytest.approx(s["wi"][2] / math.pi, rel=1e-14)
        f, _ = O.bsdf_eval(mat, wo, s["wi"])
        assert np.allclose(f, rho / math.pi, rtol=1e-14)


@pytest.mark.parametrize("name", OPAQUE + ["glass_rough"])
def test_reflection_reciprocity(O, name):
    mat = MATS[name]
    a = rng_dirs(300, 11)
    b = rng_dirs(300, 12)
    for wo, wi in zip(a, b):
        if wo[2] < 1e-4 or wi[2] < 1e-4:
            continue
        f1, _ = O.bsdf_eval(mat, wo, wi)
        f2, _ = O.bsdf_eval(mat, wi, wo)
        assert np.allclose(f1, f2, rtol=1e-12, atol=1e-300)


def test_transmission_generalised_reciprocity(O):
    # radiance-mode BTDF: f(wi -> wo side swap) = (n_i / n_o)^2 f(wo, wi), i.e. f(a,b)/n_b^2 = f(b,a)/n_a^2
    mat = M(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.35, specular_ior=1.5)
    eta = float(np.float32(1.5))
    a = rng_dirs(1000, 21)
    b = rng_dirs(1000, 22)
    n_checked = 0
    for wo, wi_up in zip(a, b):
        wi = wi_up * np.array([1, 1, -1])
        f1, _ = O.bsdf_eval(mat, wo, wi, entering=1)
        # the same pair seen from the inside: the frame flips (x, y, z) -> (x, -y, -z)
        wo2 = wi * np.array([1, -1, -1])
        wi2 = wo * np.array([1, -1, -1])
        f2, _ = O.bsdf_eval(mat, wo2, wi2, entering=0)
        if f1[0] == 0 and f2[0] == 0:
            continue
        n_checked += 1
        assert np.allclose(f2, eta * eta * f1, rtol=1e-10)
    assert n_checked > 100  # pairs with a valid refraction half-vector


def _albedo(O, mat, wo, n=6000, entering=1, eta_scale=False):
    vals = np.zeros((n, 3))
    for i in range(n):
        u = [O.uniform(9, i, 0, 1, 2), O.uniform(9, i, 0, 1, 4), O.uniform(9, i, 0, 1, 5),
             O.uniform(9, i, 0, 1, 6)]
        s = O.bsdf_sample(mat, wo, u, entering=entering)
        if s["ok"]:
            w = s["weight"]
            if eta_scale and s["refract"]:
                e = float(np.float32(mat[12]))
                w = w * (e * e if entering else 1.0 / (e * e))
            vals[i] = w
    return vals.mean(0), vals.std(0) / math.sqrt(n)


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("theta", [0.2, 1.0, 1.45])
def test_energy_bound(O, name, theta):
    # int f |cos| dwi <= 1 per channel (radiance-mode transmission rescaled by eta^2)
    mat = MATS[name]
    mean, se = _albedo(O, mat, sph(theta, 0.3), eta_scale=True)
    assert np.all(mean <= 1.0 + 4 * se + 1e-9)


def test_white_lambert_albedo_exact(O):
    mean, se = _albedo(O, MATS["lambert_white"], sph(0.7, 0.1), n=500)
    assert np.allclose(mean, 1.0, rtol=1e-14) and np.all(se < 1e-14)


def test_smooth_glass_lossless(O):
    # delta reflection + refraction: weight * (eta^2 on refraction) is exactly 1 for every sample
    mat = M(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.0, specular_ior=1.5)
    eta = float(np.float32(1.5))
    for entering in (1, 0):
        for i in range(200):
            wo = rng_dirs(1, 300 + i)[0]
            u = _u(i, 3)
            s = O.bsdf_sample(mat, wo, u, entering=entering)
            e = eta if entering else 1.0 / eta
            assert s["ok"] and s["delta"]
            w = s["weight"] * (e * e if s["refract"] else 1.0)
            assert np.allclose(w, 1.0, rtol=1e-12)
            if s["refract"]:
                # Snell's law
                si = math.hypot(wo[0], wo[1])
                st = math.hypot(s["wi"][0], s["wi"][1])
                assert abs(si - e * st) < 1e-12 and s["wi"][2] < 0


def test_delta_coat_probability(O):
    mat = MATS["coated_delta"]
    wo = sph(0.9, 0.0)
    P = O.lobe_pmf(mat, wo[2])
    ci = wo[2]
    Fc = O.fresnel_dielectric(ci, float(np.float32(1.5)))
    assert 0.0 < P[0] < 1.0 and abs(P.sum() - 1.0) < 1e-12
    n, hits = 4000, 0
    for i in range(n):
        s = O.bsdf_sample(mat, wo, [O.uniform(1, i, 0, 0, 2), 0.3, 0.6, 0.5])
        if s["delta"]:
            hits += 1
            assert np.allclose(s["weight"], Fc / P[0], rtol=1e-12)
            assert np.allclose(s["wi"], [-wo[0], -wo[1], wo[2]], atol=1e-15)
    assert abs(hits / n - P[0]) < 4 * math.sqrt(P[0] * (1 - P[0]) / n)


def _sphere_quad_pdf(O, mat, wo, entering, nt=200, npf=64):
    ct = np.polynomial.legendre.leggauss(nt)
    tot = 0.0
    for c, w in zip(*ct):
        s = math.sqrt(max(0.0, 1 - c * c))
        acc = 0.0
        for p in (np.arange(npf) + 0.5) * 2 * np.pi / npf:
            wi = np.array([s * math.cos(p), s * math.sin(p), c])
            acc += O.bsdf_eval(mat, wo, wi, entering=entering)[1]
        tot += w * acc * 2 * np.pi / npf
    return tot


@pytest.mark.parametrize("name", ["lambert", "plastic", "metal", "coated_rough", "glass_rough"])
def test_pdf_integrates_to_nondelta_mass(O, name):
    mat = MATS[name]
    wo = sph(0.6, 0.4)
    val = _sphere_quad_pdf(O, mat, wo, 1)
    P = O.lobe_pmf(mat, wo[2])
    if name == "lambert":
        assert abs(val - 1.0) < 1e-3
    else:
        # samples that leave the valid hemisphere are lost, so the mass is at most sum P_k (non-delta)
        assert val <= P.sum() + 2e-3
        assert val > 0.8 * P.sum()


@pytest.mark.parametrize("name", ["plastic", "metal_aniso", "glass_tinted", "plastic_film", "glass_film",
                                  "fuzz_plastic"])
def test_sampled_directions_chi2(O, name):
    """Histogram of sampled directions over (cos theta, phi) bins against the integrated pdf."""
    mat = MATS[name]
    wo = sph(0.8, 1.1)
    nb_c, nb_p = 8, 12
    n = 24000
    counts = np.zeros((nb_c, nb_p))
    lost = 0
    for i in range(n):
        u = [O.uniform(5, i, 0, 3, 2), O.uniform(5, i, 0, 3, 4), O.uniform(5, i, 0, 3, 5),
             O.uniform(5, i, 0, 3, 6)]
        s = O.bsdf_sample(mat, wo, u)
        if not s["ok"] or s["delta"]:
            lost += 1
            continue
        c = s["wi"][2]
        p = math.atan2(s["wi"][1], s["wi"][0]) % (2 * math.pi)
        counts[min(int((c + 1) / 2 * nb_c), nb_c - 1), min(int(p / (2 * math.pi) * nb_p), nb_p - 1)] += 1
    # expected: integrate the pdf over each bin with 16x16 Gauss points (peaked lobes need them)
    xg, wg = np.polynomial.legendre.leggauss(16)
    expect = np.zeros((nb_c, nb_p))
    for a in range(nb_c):
        c0, c1 = -1 + 2 * a / nb_c, -1 + 2 * (a + 1) / nb_c
        for b in range(nb_p):
            p0, p1 = 2 * np.pi * b / nb_p, 2 * np.pi * (b + 1) / nb_p
            acc = 0.0
            for xc, wc in zip(xg, wg):
                c = 0.5 * (c1 - c0) * xc + 0.5 * (c1 + c0)
                s_ = math.sqrt(max(0.0, 1 - c * c))
                for xp, wp in zip(xg, wg):
                    p = 0.5 * (p1 - p0) * xp + 0.5 * (p1 + p0)
                    wi = np.array([s_ * math.cos(p), s_ * math.sin(p), c])
                    acc += wc * wp * O.bsdf_eval(mat, wo, wi)[1]
            expect[a, b] = acc * 0.25 * (c1 - c0) * (p1 - p0) * n
    mask = expect > 20
    chi2 = float((((counts - expect) ** 2) / np.where(mask, expect, 1.0))[mask].sum())
    dof = int(mask.sum())
    # chi2 ~ dof +- sqrt(2 dof); allow a wide margin for the quadrature error
    assert chi2 < dof + 6 * math.sqrt(2 * dof) + 10, (chi2, dof)
    assert abs(counts[mask].sum() - expect[mask].sum()) < 0.03 * n
