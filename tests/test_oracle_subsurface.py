"""Pins of the oracle's subsurface reading (CPU only).

OpenPBR (named by the paper, Sec. 4) mixes a subsurface lobe into the
dielectric base by subsurface_weight.  The oracle takes its local limit,
where no light moves sideways under the surface: a diffuse reflector of
albedo subsurface_color, so the diffuse lobe's albedo is
rho = (1 - w) base_weight base_color + w subsurface_color (the metal keeps
base_color).  Pinned by what
follows from that definition without the code that computes it: weight 1
is the same material with base_color = subsurface_color and base_weight 1,
bit for bit, in every lobe and in the lobe choice; a metal ignores it, and
a half metal changes by half of what the same change does to a dielectric;
weight 0 ignores the subsurface colour; a Lambert base is linear in the mix; the radiance-cache
albedo inputs follow rho; and the material passes the BSDF consistency,
energy and chi-square checks of test_oracle_bsdf.py (material
"subsurface_eon").
"""
import numpy as np
import pytest

from paper_2407_19977_amd import scenes

M = scenes.material


def _dirs(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    v = r.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v[:, 2] = np.abs(v[:, 2]) + 1e-3
    return v / np.linalg.norm(v, axis=1, keepdims=True)


BASES = {
    "lambert": dict(specular_weight=0.0),
    "plastic": dict(specular_roughness=0.4),
    "rough_diffuse_coated": dict(base_diffuse_roughness=0.6, specular_roughness=0.3, coat_weight=0.7,
                                 coat_roughness=0.2),
    "weak_specular": dict(specular_weight=0.5, specular_roughness=0.25),
}


@pytest.mark.parametrize("base", list(BASES))
def test_full_weight_is_the_subsurface_colour_as_base(O, base):
    c = (0.9, 0.5, 0.3)
    a = M(base_color=(0.2, 0.7, 0.1), base_weight=0.6, subsurface_weight=1.0, subsurface_color=c, **BASES[base])
    b = M(base_color=c, base_weight=1.0, **BASES[base])
    wo, wi = _dirs(64, 1), _dirs(64, 2)
    for k in range(64):
        fa, pa = O.bsdf_eval(a, wo[k], wi[k])
        fb, pb = O.bsdf_eval(b, wo[k], wi[k])
        assert np.array_equal(fa, fb) and pa == pb
        assert np.array_equal(O.lobe_pmf(a, wo[k][2]), O.lobe_pmf(b, wo[k][2]))


def test_metal_has_no_subsurface(O):
    """Subsurface belongs to the dielectric base: a metal ignores it, and a half metal keeps
    base_color in its metal lobe (its value moves only by half the diffuse change)."""
    a = M(base_color=(0.9, 0.6, 0.3), base_metalness=1.0, specular_roughness=0.4, subsurface_weight=1.0,
          subsurface_color=(0.1, 0.9, 0.1))
    b = M(base_color=(0.9, 0.6, 0.3), base_metalness=1.0, specular_roughness=0.4)
    wo, wi = _dirs(32, 7), _dirs(32, 8)
    for k in range(32):
        assert np.array_equal(O.bsdf_eval(a, wo[k], wi[k])[0], O.bsdf_eval(b, wo[k], wi[k])[0])
    kw = dict(base_color=(0.9, 0.6, 0.3), base_metalness=0.5, specular_weight=1.0, specular_roughness=0.4)
    h0, h1 = M(**kw), M(**kw, subsurface_weight=1.0, subsurface_color=(0.1, 0.9, 0.1))
    d0 = M(base_color=(0.9, 0.6, 0.3), specular_roughness=0.4)
    d1 = M(base_color=(0.1, 0.9, 0.1), specular_roughness=0.4)
    for k in range(32):
        dh = O.bsdf_eval(h1, wo[k], wi[k])[0] - O.bsdf_eval(h0, wo[k], wi[k])[0]
        dd = O.bsdf_eval(d1, wo[k], wi[k])[0] - O.bsdf_eval(d0, wo[k], wi[k])[0]
        assert np.allclose(dh, 0.5 * dd, rtol=1e-12, atol=1e-15)


def test_zero_weight_ignores_the_subsurface_colour(O):
    a = M(base_color=(0.2, 0.7, 0.1), specular_roughness=0.4, subsurface_weight=0.0, subsurface_color=(1, 0, 1))
    b = M(base_color=(0.2, 0.7, 0.1), specular_roughness=0.4)
    wo, wi = _dirs(32, 3), _dirs(32, 4)
    for k in range(32):
        assert np.array_equal(O.bsdf_eval(a, wo[k], wi[k])[0], O.bsdf_eval(b, wo[k], wi[k])[0])


def test_lambert_base_is_linear_in_the_mix(O):
    bc, sc, w = np.array([0.2, 0.7, 0.1]), np.array([0.9, 0.5, 0.3]), 0.35
    mix = M(base_color=tuple(bc), specular_weight=0.0, subsurface_weight=w, subsurface_color=tuple(sc))
    wo, wi = _dirs(16, 5), _dirs(16, 6)
    for k in range(16):
        f, _ = O.bsdf_eval(mix, wo[k], wi[k])
        # float32 parameters, then the FP64 mix: (1 - w) bc + w sc over pi
        w32 = float(np.float32(w))
        rho = (1.0 - w32) * bc.astype(np.float32).astype(np.float64) + w32 * sc.astype(np.float32).astype(np.float64)
        assert np.allclose(f, rho / np.pi, rtol=1e-14, atol=0.0)


def test_cache_albedo_inputs_follow_the_mix(O):
    m = M(base_color=(0.2, 0.6, 1.0), base_weight=0.5, transmission_weight=0.0, specular_roughness=0.4,
          subsurface_weight=0.5, subsurface_color=(0.8, 0.4, 0.0))
    x = O.nrc_inputs((0, 0, 0), (1, 1, 1), (0.5, 0.5, 0.5), (0, 0, 1), (0, 0, 1), m)
    # (1 - 0.5) 0.5 (0.2, 0.6, 1.0) + 0.5 (0.8, 0.4, 0.0)
    assert np.allclose(x[8:11], [0.45, 0.35, 0.25], atol=1e-7)
