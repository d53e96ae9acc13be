"""Pins of the oracle's thin film on the dielectric interface (CPU only).

OpenPBR (named by the paper, Sec. 4) puts an optional thin film on the
specular interface.  The oracle's reflectance of the stack (incident medium
| film | base) is the Airy sum of the film's multiply reflected waves; it is
pinned here by what the optics fixes independently of that formula: a film
of zero thickness, or one whose index matches either neighbour, leaves the
bare interface's Fresnel reflectance; a quarter-wave layer of index sqrt(n)
cancels the reflection at normal incidence, and any quarter-wave layer
reflects ((n3 - n2^2) / (n3 + n2^2))^2 there; a half-wave layer is absent;
the reflectance is periodic in the thickness with period
lambda / (2 n_film cos_film); it is the same seen from either side of the
stack (Stokes reciprocity); total internal reflection reflects everything.
The BSDF with a film is then checked like every other material: weight =
f |cos| / pdf, reciprocity, energy, and a film of zero thickness reproducing
the bare material.
"""
import math

import numpy as np
import pytest

from paper_2407_19977_amd import scenes

M = scenes.material
ANGLES = [1.0, 0.93, 0.71, 0.42, 0.13, 0.02]


@pytest.mark.parametrize("n2", [1.2, 1.38, 2.0])
@pytest.mark.parametrize("n3", [1.5, 1.1, 1.0 / 1.5, 2.4])
def test_zero_thickness_is_the_bare_interface(O, n2, n3):
    for c in ANGLES:
        want = O.fresnel_dielectric(c, n3)
        for lam in (450.0, 650.0):
            assert O.film_reflectance(c, n2, n3, n2, 0.0, lam) == pytest.approx(want, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("d", [37.0, 250.0, 1234.5])
def test_index_matched_film_is_invisible(O, d):
    for n3 in (1.5, 0.8, 2.2):
        for c in ANGLES:
            want = O.fresnel_dielectric(c, n3)
            # film index equal to the incident medium's, then to the base's
            assert O.film_reflectance(c, 1.0, n3, 1.0, d, 550.0) == pytest.approx(want, rel=1e-12, abs=1e-15)
            if n3 >= 1.0:
                assert O.film_reflectance(c, n3, n3, n3, d, 550.0) == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_quarter_wave_antireflection(O):
    n3 = 1.52
    n2 = math.sqrt(n3)
    for lam in (450.0, 550.0, 650.0):
        d = lam / (4.0 * n2)
        assert O.film_reflectance(1.0, n2, n3, n2, d, lam) < 1e-14
        # away from its design wavelength the coating reflects again, less than the bare glass
        r = O.film_reflectance(1.0, n2, n3, n2, d, lam * 1.3)
        assert 0.0 < r < O.fresnel_dielectric(1.0, n3)


@pytest.mark.parametrize("n2,n3", [(1.38, 1.52), (2.1, 1.5), (1.7, 1.0 / 1.33)])
def test_quarter_and_half_wave_closed_forms(O, n2, n3):
    lam = 520.0
    quarter = O.film_reflectance(1.0, n2, n3, n2, lam / (4.0 * n2), lam)
    assert quarter == pytest.approx(((n3 - n2 * n2) / (n3 + n2 * n2)) ** 2, rel=1e-12, abs=1e-15)
    half = O.film_reflectance(1.0, n2, n3, n2, lam / (2.0 * n2), lam)
    assert half == pytest.approx(((1.0 - n3) / (1.0 + n3)) ** 2, rel=1e-12, abs=1e-15)


def test_periodic_in_thickness(O):
    n2, n3, lam = 1.33, 1.6, 480.0
    for c in ANGLES:
        c2 = math.sqrt(1.0 - (1.0 - c * c) / (n2 * n2))
        period = lam / (2.0 * n2 * c2)
        for d in (10.0, 333.0):
            a = O.film_reflectance(c, n2, n3, n2, d, lam)
            b = O.film_reflectance(c, n2, n3, n2, d + 3 * period, lam)
            assert a == pytest.approx(b, rel=1e-9, abs=1e-15)


def test_same_reflectance_from_either_side(O):
    """Stokes: stack 1 | n2 | n3 at incidence c1 reflects as much as n3 | n2 | 1 at the refracted angle."""
    n2, n3, d, lam = 1.4, 1.55, 310.0, 600.0
    for c1 in ANGLES[:-1]:
        s1 = math.sqrt(1.0 - c1 * c1)
        c3 = math.sqrt(1.0 - (s1 / n3) ** 2)
        fwd = O.film_reflectance(c1, n2, n3, n2, d, lam)
        back = O.film_reflectance(c3, n2 / n3, 1.0 / n3, n2, d, lam)
        assert fwd == pytest.approx(back, rel=1e-11)


def test_total_internal_reflection(O):
    # leaving glass (relative exit index 1/1.5) beyond the critical angle, with a film of index 1.3
    n3 = 1.0 / 1.5
    crit = math.sqrt(1.0 - n3 * n3)  # cos of the critical angle
    for c in (0.5 * crit, 0.1 * crit, 0.0):
        assert O.film_reflectance(c, 1.3 / 1.5, n3, 1.3, 200.0, 550.0) == 1.0
    r = O.film_reflectance(min(1.0, 1.2 * crit), 1.3 / 1.5, n3, 1.3, 200.0, 550.0)
    assert 0.0 < r < 1.0


def test_bounded_and_coloured(O):
    rng = np.random.Generator(np.random.PCG64(5))
    vals = []
    for _ in range(2000):
        c = rng.uniform(0.0, 1.0)
        n2 = rng.uniform(1.0, 2.5)
        n3 = rng.uniform(0.5, 2.5)
        d = rng.uniform(0.0, 2000.0)
        r = O.film_reflectance(c, n2, n3, n2, d, rng.uniform(400.0, 700.0))
        assert 0.0 <= r <= 1.0
        vals.append(r)
    # interference: the three channels of one film differ
    F = [O.film_reflectance(1.0, 1.33, 1.5, 1.33, 400.0, lam) for lam in (650.0, 550.0, 450.0)]
    assert max(F) - min(F) > 0.02


FILM_MATS = {
    "plastic_film": M(base_color=(0.5, 0.3, 0.2), specular_roughness=0.4, thin_film_weight=1.0,
                      thin_film_thickness=0.35, thin_film_ior=1.33),
    "plastic_film_half": M(base_color=(0.2, 0.5, 0.3), specular_roughness=0.25, base_diffuse_roughness=0.5,
                           thin_film_weight=0.5, thin_film_thickness=0.8, thin_film_ior=2.0),
    "glass_film": M(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.3, specular_ior=1.5,
                    thin_film_weight=1.0, thin_film_thickness=0.5, thin_film_ior=1.38),
}


def _dirs(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    v = r.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v[:, 2] = np.abs(v[:, 2])
    return v


@pytest.mark.parametrize("name", list(FILM_MATS))
def test_film_sample_weight_is_f_cos_over_pdf(O, name):
    mat = FILM_MATS[name]
    n_ok = 0
    for i, wo in enumerate(_dirs(200, 3)):
        if wo[2] < 1e-3:
            continue
        u = [O.uniform(7, i, 0, 0, 2), O.uniform(7, i, 0, 0, 4), O.uniform(7, i, 0, 0, 5), O.uniform(7, i, 0, 0, 6)]
        s = O.bsdf_sample(mat, wo, u)
        if not s["ok"] or s["delta"]:
            continue
        f, pdf = O.bsdf_eval(mat, wo, s["wi"])
        assert pdf == pytest.approx(s["pdf"], rel=1e-12)
        assert np.allclose(s["weight"], f * abs(s["wi"][2]) / pdf, rtol=1e-10)
        n_ok += 1
    assert n_ok > 100


@pytest.mark.parametrize("name", ["plastic_film", "plastic_film_half"])
def test_film_reflection_reciprocity(O, name):
    mat = FILM_MATS[name]
    for wo, wi in zip(_dirs(200, 11), _dirs(200, 12)):
        if wo[2] < 1e-4 or wi[2] < 1e-4:
            continue
        f1, _ = O.bsdf_eval(mat, wo, wi)
        f2, _ = O.bsdf_eval(mat, wi, wo)
        assert np.allclose(f1, f2, rtol=1e-12, atol=1e-300)


def test_zero_thickness_film_reproduces_the_bare_material(O):
    for base in (dict(base_color=(0.5, 0.3, 0.2), specular_roughness=0.4),
                 dict(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.3, specular_ior=1.45)):
        bare = M(**base)
        film = M(**base, thin_film_weight=1.0, thin_film_thickness=0.0, thin_film_ior=1.8)
        for entering in (1, 0):
            for wo, wi in zip(_dirs(100, 21), _dirs(100, 22)):
                for w in (wi, wi * np.array([1, 1, -1])):
                    f1, p1 = O.bsdf_eval(bare, wo, w, entering=entering)
                    f2, p2 = O.bsdf_eval(film, wo, w, entering=entering)
                    assert np.allclose(f1, f2, rtol=1e-12, atol=1e-300) and p1 == pytest.approx(p2, rel=1e-12)


def test_smooth_film_on_glass_conserves_energy(O):
    """Delta reflection and refraction through a film: each channel reflects its film reflectance
    F_c and refracts 1 - F_c, whatever probability picks between them, so the expected weight
    (refraction rescaled by eta^2) is exactly 1 per channel."""
    f32 = lambda v: float(np.float32(v))
    ior, fior, d_um = f32(1.5), f32(1.35), f32(0.45)
    mat = M(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.0, specular_ior=1.5,
            thin_film_weight=1.0, thin_film_thickness=0.45, thin_film_ior=1.35)
    wo = np.array([0.3, 0.1, 0.0])
    wo[2] = math.sqrt(1.0 - wo[0] ** 2 - wo[1] ** 2)
    for entering in (1, 0):
        e = ior if entering else 1.0 / ior
        n2 = fior if entering else fior / ior
        F = np.array([O.film_reflectance(wo[2], n2, e, fior, 1000.0 * d_um, lam) for lam in (650.0, 550.0, 450.0)])
        pr = 0.2126 * F[0] + 0.7152 * F[1] + 0.0722 * F[2]  # reflect-vs-refract: the luminance (tw = 1)
        P = O.lobe_pmf(mat, wo[2], entering=entering)
        refl = O.bsdf_sample(mat, wo, [0.5, 0.5, 0.5, 0.0], entering=entering)
        refr = O.bsdf_sample(mat, wo, [0.5, 0.5, 0.5, 0.999999], entering=entering)
        assert refl["ok"] and refl["delta"] and not refl["refract"]
        assert refr["ok"] and refr["delta"] and refr["refract"]
        assert np.allclose(refl["weight"], F / (P[2] * pr), rtol=1e-12)
        assert np.allclose(refr["weight"] * e * e, (1.0 - F) / (P[2] * (1.0 - pr)), rtol=1e-12)
        expected = P[2] * (pr * refl["weight"] + (1.0 - pr) * refr["weight"] * e * e)
        assert np.allclose(expected, 1.0, rtol=1e-12)
        assert np.ptp(F) > 1e-3  # the film colours the reflection
