"""Pins of the oracle's light sampling and ray/triangle geometry (CPU only).

Lights: solid angles of a rectangle and a triangle in closed form, the
environment pdf's normalisation and its texel histogram, and the irradiance
of a uniform sky.  Geometry (Sec. 5.1.1, AABB BVH): the BVH answer equals
brute force, the single-precision watertight test leaks no ray out of a
closed mesh, ties resolve to the smallest id and degenerate triangles are
never hit.
"""
import math

import numpy as np
import pytest

from paper_2407_19977_amd import scenes


def _scene(meshes_tris, mats, env=None, instances=()):
    """Build a duck-typed scene from a list of (vertices, indices, material_ids)."""
    ms = [scenes.Mesh(np.asarray(v, np.float32), np.asarray(i, np.int32), np.asarray(m, np.int32))
          for v, i, m in meshes_tris]
    cam = scenes.Camera((0, 0, -3), (0, 0, 0), (0, 1, 0), 40.0, 8, 8)
    return scenes.Scene("t", ms, list(instances), np.stack(mats), env, cam, 1, 1)


def _quad_light(a, b, d, L=5.0):
    """a x b rectangle in the plane y = d centred on the y axis, emitting toward -y."""
    v = np.array([[-a / 2, d, -b / 2], [a / 2, d, -b / 2], [a / 2, d, b / 2], [-a / 2, d, b / 2]])
    # winding so that cross(v1-v0, v2-v0) points to -y
    idx = np.array([[0, 1, 2], [0, 2, 3]])
    n = np.cross(v[1] - v[0], v[2] - v[0])
    if n[1] > 0:
        idx = idx[:, ::-1]
    emis = scenes.material(base_weight=0.0, specular_weight=0.0, emission_luminance=L)
    return v, idx, [0, 0], emis


def test_rectangle_solid_angle(O):
    a, b, d = 0.8, 0.5, 0.7
    v, i, m, emis = _quad_light(a, b, d)
    os_ = O.OracleScene(_scene([(v, i, m)], [emis]))
    assert os_.n_lights == 2
    n = 40000
    inv = np.empty(n)
    for k in range(n):
        s = os_.sample_light([0, 0, 0], O.uniform(1, k, 0, 0, 7), O.uniform(1, k, 0, 0, 8), O.uniform(1, k, 0, 0, 9))
        assert s["ok"] and s["light"] in (0, 1)
        assert np.allclose(s["Le"], 5.0)
        inv[k] = 1.0 / s["pdf"]
    af, bf, df = (float(np.float32(x)) for x in (a, b, d))
    omega = 4 * math.asin(af * bf / math.sqrt((af * af + 4 * df * df) * (bf * bf + 4 * df * df)))
    assert abs(inv.mean() - omega) < 4 * inv.std() / math.sqrt(n) + 1e-9


def test_triangle_solid_angle_off_axis(O):
    # Van Oosterom & Strackee: tan(omega/2) = |a.(b x c)| / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|)
    tri = np.array([[0.3, 1.0, -0.2], [1.1, 1.4, 0.1], [0.2, 0.9, 0.9]], dtype=np.float32)
    if np.cross(tri[1] - tri[0], tri[2] - tri[0])[1] > 0:
        tri = tri[[0, 2, 1]]
    emis = scenes.material(base_weight=0.0, specular_weight=0.0, emission_luminance=2.0)
    os_ = O.OracleScene(_scene([(tri, [[0, 1, 2]], [0])], [emis]))
    p = np.array([0.1, -0.2, 0.05])
    A, B, C = (tri.astype(np.float64) - p)
    la, lb, lc = np.linalg.norm(A), np.linalg.norm(B), np.linalg.norm(C)
    num = abs(A @ np.cross(B, C))
    den = la * lb * lc + (A @ B) * lc + (A @ C) * lb + (B @ C) * la
    omega = 2 * math.atan2(num, den)
    n = 40000
    inv = np.array([1.0 / os_.sample_light(p, 0.5, O.uniform(2, k, 0, 0, 8), O.uniform(2, k, 0, 0, 9))["pdf"]
                    for k in range(n)])
    assert abs(inv.mean() - omega) < 4 * inv.std() / math.sqrt(n) + 1e-9


def test_light_selection_proportional_to_power(O):
    v1, i1, _, e1 = _quad_light(0.5, 0.5, 1.0, L=3.0)
    v2 = v1 + np.array([2.0, 0, 0])
    e2 = scenes.material(base_weight=0.0, specular_weight=0.0, emission_luminance=1.0,
                         emission_color=(1.0, 0.5, 0.25))
    os_ = O.OracleScene(_scene([(np.concatenate([v1, v2]), np.concatenate([i1, i1 + 4]), [0, 0, 1, 1])], [e1, e2]))
    lum2 = 0.2126 * 1.0 + 0.7152 * 0.5 + 0.0722 * 0.25
    p_first = 3.0 / (3.0 + lum2)  # equal areas: selection follows luminance x area
    n = 20000
    first = sum(os_.sample_light([0, 0, 0], O.uniform(4, k, 0, 0, 7), 0.3, 0.3)["light"] < 2 for k in range(n))
    assert abs(first / n - p_first) < 4 * math.sqrt(p_first * (1 - p_first) / n)


def _env_scene(env):
    tri = np.array([[100, 100, 100], [100.1, 100, 100], [100, 100.1, 100]], dtype=np.float32)
    return _scene([(tri, [[0, 1, 2]], [0])], [scenes.lambert((0.5, 0.5, 0.5))], env=env)


def _hot_env(w=64, h=32):
    r = np.random.Generator(np.random.PCG64(5))
    env = r.uniform(0.1, 1.0, size=(h, w, 3)).astype(np.float32)
    env[9, 40] = (500.0, 400.0, 300.0)
    env[0, :] = 0.0  # a black row must never be sampled
    return env


def test_env_pdf_normalised(O):
    env = _hot_env()
    h, w = env.shape[:2]
    os_ = O.OracleScene(_env_scene(env))
    # the pdf times sin(theta) is constant inside a texel, so the centre rule is exact
    tot = 0.0
    for r in range(h):
        th = math.pi * (r + 0.5) / h
        for c in range(w):
            ph = 2 * math.pi * ((c + 0.5) / w - 0.5)
            d = [math.sin(th) * math.sin(ph), math.cos(th), -math.sin(th) * math.cos(ph)]
            tot += os_.env_pdf(d) * math.sin(th) * (math.pi / h) * (2 * math.pi / w)
            assert np.allclose(os_.env_radiance(d), env[r, c])
    assert abs(tot - 1.0) < 1e-12


def test_env_sampling_histogram_and_pdf(O):
    env = _hot_env()
    h, w = env.shape[:2]
    os_ = O.OracleScene(_env_scene(env))
    lum = 0.2126 * env[..., 0].astype(np.float64) + 0.7152 * env[..., 1] + 0.0722 * env[..., 2]
    wts = lum * np.sin(np.pi * (np.arange(h) + 0.5) / h)[:, None]
    P = wts / wts.sum()
    n = 60000
    counts = np.zeros(h * w)
    for k in range(n):
        s = os_.sample_light([0, 0, 0], 0.1, O.uniform(6, k, 0, 0, 8), O.uniform(6, k, 0, 0, 9))
        assert s["ok"] and s["light"] >= 0x80000000
        t = s["light"] - 0x80000000
        counts[t] += 1
        assert np.allclose(s["Le"], env.reshape(-1, 3)[t])
        # returned pdf = environment density of the sampled direction (selection probability 1 here)
        assert s["pdf"] == pytest.approx(os_.env_pdf(s["wl"]), rel=1e-6)
    assert counts.reshape(h, w)[0].sum() == 0
    e = P.reshape(-1) * n
    m = e > 10
    chi2 = float((((counts - e) ** 2) / np.where(m, e, 1))[m].sum())
    dof = int(m.sum())
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_uniform_sky_irradiance(O):
    # E[L max(0, n.w) / pdf] = pi L for the upper-hemisphere normal n = +y
    env = scenes.uniform_env(1.7, 48, 24)
    os_ = O.OracleScene(_env_scene(env))
    n = 40000
    v = np.empty(n)
    for k in range(n):
        s = os_.sample_light([0, 0, 0], 0.2, O.uniform(8, k, 0, 0, 8), O.uniform(8, k, 0, 0, 9))
        v[k] = s["Le"][1] * max(0.0, s["wl"][1]) / s["pdf"]
    L = float(np.float32(1.7))
    assert abs(v.mean() - math.pi * L) < 4 * v.std() / math.sqrt(n)


# ------------------------------------------------------------- geometry --

def _soup(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    c = r.uniform(-1, 1, size=(n, 1, 3))
    v = (c + 0.15 * r.normal(size=(n, 3, 3))).reshape(-1, 3)
    return v, np.arange(3 * n).reshape(n, 3)


def _rays(n, seed, box=1.5):
    r = np.random.Generator(np.random.PCG64(seed))
    o = r.uniform(-box, box, size=(n, 3))
    d = r.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


@pytest.mark.parametrize("which", ["soup", "cornell", "icosphere"])
def test_bvh_equals_brute_force_f64(O, which):
    if which == "soup":
        v, i = _soup(3000, 1)
        sc = _scene([(v, i, np.zeros(len(i)))], [scenes.lambert((0.5, 0.5, 0.5))])
    elif which == "cornell":
        sc = scenes.cornell()
    else:
        v, f = scenes.icosphere(3)
        sc = _scene([(v, f, np.zeros(len(f)))], [scenes.lambert((0.5, 0.5, 0.5))])
    os_ = O.OracleScene(sc)
    o, d = _rays(3000, 2)
    if which == "cornell":
        o = o * 0.3 + 0.5
    n_hit = 0
    for k in range(len(o)):
        a = os_.closest(o[k], d[k])
        b = os_.closest(o[k], d[k], brute=True)
        assert a[0] == b[0]
        if a[0]:
            n_hit += 1
            assert a[1:] == b[1:]
    assert n_hit > 300


def test_watertight_f32_closed_mesh(O):
    """Rays from inside a closed icosphere, including rays aimed exactly at its
    vertices and edge midpoints, always hit it in single precision."""
    v, f = scenes.icosphere(3)
    v = (v * 2.0 + np.array([0.3, -0.2, 0.1])).astype(np.float32)
    os_ = O.OracleScene(_scene([(v, f, np.zeros(len(f)))], [scenes.lambert((0.5, 0.5, 0.5))]))
    r = np.random.Generator(np.random.PCG64(3))
    origins = [np.array([0.3, -0.2, 0.1], np.float32)] + [
        (np.array([0.3, -0.2, 0.1]) + r.uniform(-0.8, 0.8, 3)).astype(np.float32) for _ in range(7)]
    targets = np.concatenate([v.astype(np.float64), 0.5 * (v[f[:, 0]].astype(np.float64) + v[f[:, 1]]),
                              r.normal(size=(4000, 3)) * 5.0])
    rays = []
    for o in origins:
        d = targets - o.astype(np.float64)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rr = np.zeros((len(d), 8), np.float32)
        rr[:, 0:3] = o
        rr[:, 3] = 0.0
        rr[:, 4:7] = d
        rr[:, 7] = np.inf
        rays.append(rr)
    rays = np.concatenate(rays)
    hits = os_.closest_f32(rays)
    assert hits[:, 5].all(), f"{int((hits[:, 5] == 0).sum())} rays escaped"


def test_f32_ties_and_degenerates(O):
    # two identical triangles: the lower primitive id wins; a zero-area triangle is never hit
    tri = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], np.float32)
    deg = np.array([[-1, 0, -0.5], [1, 0, -0.5], [0, 0, -0.5]], np.float32)  # collinear
    v = np.concatenate([deg, tri, tri])
    sc = _scene([(v, [[0, 1, 2], [3, 4, 5], [6, 7, 8]], [0, 0, 0])], [scenes.lambert((0.5, 0.5, 0.5))])
    os_ = O.OracleScene(sc)
    rays = np.array([[0.01, 0.0, -2.0, 0.0, 0.0, 0.0, 1.0, np.inf],
                     [0.0, 0.0, -2.0, 0.0, 0.0, 0.0, 1.0, np.inf]], np.float32)
    h = os_.closest_f32(rays)
    assert list(h[:, 2]) == [1, 1] and h[:, 5].all()
    assert np.frombuffer(h[0, 0].tobytes(), np.float32)[0] == np.float32(2.0)


def test_f32_agrees_with_f64_almost_everywhere(O):
    v, i = _soup(2000, 4)
    sc = _scene([(v, i, np.zeros(len(i)))], [scenes.lambert((0.5, 0.5, 0.5))])
    os_ = O.OracleScene(sc)
    o, d = _rays(4000, 5)
    rays = np.zeros((len(o), 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 4:7] = d
    rays[:, 3] = 0.0
    rays[:, 7] = np.inf
    h32 = os_.closest_f32(rays)
    agree = 0
    for k in range(len(o)):
        a = os_.closest(rays[k, 0:3].astype(np.float64), rays[k, 4:7].astype(np.float64), tmin=0.0)
        if (a[0] and h32[k, 5] and a[5] == h32[k, 2]) or (not a[0] and not h32[k, 5]):
            agree += 1
    assert agree >= len(o) - 4
