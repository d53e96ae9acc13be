"""Seeded synthetic scenes: the input data for both the HIP path tracer and the oracle.

This module holds geometry, material parameters, environment texels and
camera set-ups only.  It contains none of the light-transport arithmetic
(no intersection, BSDF, sampling or integration), so the HIP path and the
FP64 oracle can both read the same inputs without sharing any method code.

The paper renders proprietary CAD models (Sec. 5.2 and App. A, Table 2:
pushbutton LODs of 1,068,735 / 106,873 / 10,687 triangles) that are not
available; the scenes below are synthetic stand-ins of the same shape:

* ``cornell()``      closed-box scene, 36 triangles, one quad area light.
* ``spheres()``      ~1.31M triangles: 64 noise-displaced level-5 icospheres
                     on a ground plane, metal / coated-diffuse mix, sky
                     environment with a 0.5 degree sun.
* ``instanced()``    ~10.8M instanced triangles: 400 instances of 5 bevelled
                     cylinder / torus meshes in a two-level hierarchy.
* furnace / plane / glass test scenes with closed-form answers.

Materials use the OpenPBR parameter names (Sec. 4 lists the parameter
families); every record is a row of ``MATERIAL_DTYPE``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# One OpenPBR parameter record: 39 float32, in this order.  The C ABI's
# pt_openpbr_material and the oracle's input record have the same layout.
MATERIAL_FIELDS = [
    ("base_weight", 1), ("base_color", 3), ("base_metalness", 1),
    ("base_diffuse_roughness", 1),
    ("specular_weight", 1), ("specular_color", 3), ("specular_roughness", 1),
    ("specular_roughness_anisotropy", 1), ("specular_ior", 1),
    ("transmission_weight", 1), ("transmission_color", 3),
    ("coat_weight", 1), ("coat_color", 3), ("coat_roughness", 1), ("coat_ior", 1),
    ("emission_luminance", 1), ("emission_color", 3),
    ("thin_film_weight", 1), ("thin_film_thickness", 1), ("thin_film_ior", 1),
    ("fuzz_weight", 1), ("fuzz_color", 3), ("fuzz_roughness", 1),
    ("subsurface_weight", 1), ("subsurface_color", 3),
]
MATERIAL_FLOATS = sum(n for _, n in MATERIAL_FIELDS)  # 39


def material(**kw) -> np.ndarray:
    """Return one material as float32[39], OpenPBR defaults for unset fields.

    Defaults follow the OpenPBR specification: base_weight 1, base_color 0.8,
    specular_weight 1, specular_color 1, specular_roughness 0.3,
    specular_ior 1.5, transmission_color 1, coat_color 1, coat_ior 1.6,
    emission_color 1, thin_film_thickness 0.5 (micrometres), thin_film_ior
    1.5, fuzz_color 1, fuzz_roughness 0.5, subsurface_color 0.8, everything
    else 0.
    """
    d = {
        "base_weight": 1.0, "base_color": (0.8, 0.8, 0.8), "base_metalness": 0.0,
        "base_diffuse_roughness": 0.0,
        "specular_weight": 1.0, "specular_color": (1.0, 1.0, 1.0),
        "specular_roughness": 0.3, "specular_roughness_anisotropy": 0.0,
        "specular_ior": 1.5,
        "transmission_weight": 0.0, "transmission_color": (1.0, 1.0, 1.0),
        "coat_weight": 0.0, "coat_color": (1.0, 1.0, 1.0), "coat_roughness": 0.0,
        "coat_ior": 1.6,
        "emission_luminance": 0.0, "emission_color": (1.0, 1.0, 1.0),
        "thin_film_weight": 0.0, "thin_film_thickness": 0.5, "thin_film_ior": 1.5,
        "fuzz_weight": 0.0, "fuzz_color": (1.0, 1.0, 1.0), "fuzz_roughness": 0.5,
        "subsurface_weight": 0.0, "subsurface_color": (0.8, 0.8, 0.8),
    }
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown OpenPBR parameter {k!r}")
        d[k] = v
    out = []
    for name, n in MATERIAL_FIELDS:
        v = d[name]
        if n == 1:
            out.append(float(v))
        else:
            v = tuple(float(x) for x in v)
            assert len(v) == n
            out.extend(v)
    return np.asarray(out, dtype=np.float32)


def lambert(albedo) -> np.ndarray:
    """Base-only Lambertian: no specular layer (specular_weight 0)."""
    return material(base_color=tuple(albedo), specular_weight=0.0)


@dataclasses.dataclass
class Mesh:
    vertices: np.ndarray      # float32 [n_vertices, 3]
    indices: np.ndarray       # int32 [n_triangles, 3]
    material_ids: np.ndarray  # int32 [n_triangles]

    @property
    def n_triangles(self) -> int:
        return int(self.indices.shape[0])


@dataclasses.dataclass
class Instance:
    object_to_world: np.ndarray  # float32 [3, 4], rigid (rotation | translation)
    mesh: int
    material_override: int = -1


@dataclasses.dataclass
class Camera:
    eye: tuple
    look_at: tuple
    up: tuple
    vfov_deg: float
    width: int
    height: int


@dataclasses.dataclass
class Scene:
    name: str
    meshes: List[Mesh]
    instances: List[Instance]          # empty: single level, meshes in world space
    materials: np.ndarray              # float32 [n_materials, 39]
    env: Optional[np.ndarray]          # float32 [h, w, 3] equirect (y up) or None
    camera: Camera
    spp: int
    max_depth: int
    seed: int = 0

    @property
    def n_triangles(self) -> int:
        if not self.instances:
            return sum(m.n_triangles for m in self.meshes)
        return sum(self.meshes[i.mesh].n_triangles for i in self.instances)

    def with_camera(self, **kw) -> "Scene":
        cam = dataclasses.replace(self.camera, **kw)
        return dataclasses.replace(self, camera=cam)


# --------------------------------------------------------------------------
# geometry helpers (data generation only)
# --------------------------------------------------------------------------

def _quad(p0, p1, p2, p3, normal):
    """Two triangles (p0,p1,p2), (p0,p2,p3) wound so cross(v1-v0, v2-v0) points along `normal`."""
    p = np.asarray([p0, p1, p2, p3], dtype=np.float64)
    n = np.cross(p[1] - p[0], p[2] - p[0])
    if np.dot(n, normal) < 0:
        p = p[[0, 3, 2, 1]]
    return p, np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)


def _box_faces(lo, hi, outward=True):
    """Six quads of an axis-aligned box, normals outward (or inward)."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    s = 1.0 if outward else -1.0
    faces = [
        ([x0, y0, z0], [x1, y0, z0], [x1, y0, z1], [x0, y0, z1], [0, -s, 0]),  # bottom
        ([x0, y1, z0], [x1, y1, z0], [x1, y1, z1], [x0, y1, z1], [0, s, 0]),   # top
        ([x0, y0, z0], [x0, y1, z0], [x0, y1, z1], [x0, y0, z1], [-s, 0, 0]),  # -x
        ([x1, y0, z0], [x1, y1, z0], [x1, y1, z1], [x1, y0, z1], [s, 0, 0]),   # +x
        ([x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0], [0, 0, -s]),  # -z
        ([x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1], [0, 0, s]),   # +z
    ]
    return faces


class _MeshBuilder:
    def __init__(self):
        self.v = []
        self.i = []
        self.m = []
        self.nv = 0

    def add(self, verts, idx, mat):
        verts = np.asarray(verts, dtype=np.float64)
        idx = np.asarray(idx, dtype=np.int64)
        self.v.append(verts)
        self.i.append(idx + self.nv)
        self.m.append(np.full(idx.shape[0], mat, dtype=np.int32))
        self.nv += verts.shape[0]

    def add_quad(self, p0, p1, p2, p3, normal, mat):
        p, idx = _quad(p0, p1, p2, p3, normal)
        self.add(p, idx, mat)

    def mesh(self) -> Mesh:
        return Mesh(np.concatenate(self.v).astype(np.float32),
                    np.concatenate(self.i).astype(np.int32),
                    np.concatenate(self.m).astype(np.int32))


# --------------------------------------------------------------------------
# closed box scene (36 triangles)
# --------------------------------------------------------------------------

def cornell(width=128, height=128, spp=16, max_depth=4, seed=0) -> Scene:
    """Closed box [0,1]^3 open at z=0: floor, ceiling, back, left, right walls
    (inward normals), cube A [.15,.45]x[0,.30]x[.15,.45], cube B
    [.55,.85]x[0,.60]x[.50,.80] (outward normals) and a 0.2x0.2 quad light at
    y=0.999 facing -y with radiance 15.  34 diffuse triangles + 2 emissive.

    Albedos: per object and per channel U[0.2,0.8] from PCG64(0), drawn in
    the order floor, ceiling, back, left, right, cubeA, cubeB.
    """
    rng = np.random.Generator(np.random.PCG64(0))
    alb = rng.uniform(0.2, 0.8, size=(7, 3))
    mats = [lambert(a) for a in alb]
    mats.append(material(base_weight=0.0, specular_weight=0.0,
                         emission_luminance=15.0, emission_color=(1.0, 1.0, 1.0)))
    b = _MeshBuilder()
    b.add_quad([0, 0, 0], [1, 0, 0], [1, 0, 1], [0, 0, 1], [0, 1, 0], 0)    # floor
    b.add_quad([0, 1, 0], [1, 1, 0], [1, 1, 1], [0, 1, 1], [0, -1, 0], 1)   # ceiling
    b.add_quad([0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1], [0, 0, -1], 2)   # back
    b.add_quad([0, 0, 0], [0, 1, 0], [0, 1, 1], [0, 0, 1], [1, 0, 0], 3)    # left
    b.add_quad([1, 0, 0], [1, 1, 0], [1, 1, 1], [1, 0, 1], [-1, 0, 0], 4)   # right
    for f in _box_faces([.15, 0, .15], [.45, .30, .45]):
        b.add_quad(*f, 5)
    for f in _box_faces([.55, 0, .50], [.85, .60, .80]):
        b.add_quad(*f, 6)
    b.add_quad([.4, .999, .4], [.6, .999, .4], [.6, .999, .6], [.4, .999, .6], [0, -1, 0], 7)
    cam = Camera((0.5, 0.5, -1.4), (0.5, 0.5, 0.0), (0.0, 1.0, 0.0), 40.0, width, height)
    return Scene("cornell", [b.mesh()], [], np.stack(mats), None, cam, spp, max_depth, seed)


# --------------------------------------------------------------------------
# material zoo: every shading class, mixed and tinted OpenPBR materials
# --------------------------------------------------------------------------

ZOO_MATERIALS = [
    # (name, OpenPBR parameters)
    ("partial metal", dict(base_metalness=0.5, base_color=(0.9, 0.6, 0.3), specular_color=(0.8, 0.9, 1.0),
                           specular_roughness=0.3)),
    ("coat over metal", dict(base_metalness=1.0, base_color=(0.95, 0.8, 0.5), specular_roughness=0.25,
                             coat_weight=1.0, coat_roughness=0.1, coat_color=(0.9, 0.8, 1.0), coat_ior=1.5)),
    ("delta coat over anisotropic metal", dict(base_metalness=1.0, base_color=(0.7, 0.8, 0.9), specular_roughness=0.4,
                                              specular_roughness_anisotropy=0.6, coat_weight=0.6,
                                              coat_roughness=0.0, coat_color=(1.0, 0.85, 0.85))),
    ("transmission over partial metal", dict(base_metalness=0.3, base_color=(0.8, 0.7, 0.6), specular_roughness=0.2,
                                             transmission_weight=0.5, transmission_color=(0.8, 1.0, 0.9))),
    ("transmission over diffuse", dict(transmission_weight=0.7, base_color=(0.6, 0.3, 0.2), specular_roughness=0.25,
                                       transmission_color=(0.7, 0.9, 0.8), specular_ior=1.45)),
    ("weak tinted specular plastic, half subsurface", dict(base_color=(0.2, 0.5, 0.3), specular_weight=0.6,
                                                           specular_color=(1.0, 0.7, 0.7), specular_roughness=0.3,
                                                           subsurface_weight=0.5,
                                                           subsurface_color=(0.9, 0.7, 0.5))),
    ("anisotropic coated plastic", dict(base_color=(0.3, 0.3, 0.7), specular_roughness=0.35,
                                        specular_roughness_anisotropy=0.6, coat_weight=0.5, coat_roughness=0.2,
                                        coat_color=(1.0, 0.9, 0.7), coat_ior=1.6)),
    ("weak tinted metal", dict(base_metalness=1.0, base_weight=0.9, base_color=(0.95, 0.9, 0.8), specular_weight=0.7,
                               specular_color=(0.6, 0.8, 1.0), specular_roughness=0.15)),
    ("thin film on plastic", dict(base_color=(0.15, 0.15, 0.2), specular_roughness=0.15, thin_film_weight=1.0,
                                  thin_film_thickness=0.38, thin_film_ior=1.33)),
    ("thin film on smooth glass", dict(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.0,
                                       thin_film_weight=1.0, thin_film_thickness=0.3, thin_film_ior=1.38)),
    ("half-weight thin film on rough glass", dict(base_weight=0.0, transmission_weight=1.0, specular_roughness=0.3,
                                                  thin_film_weight=0.5, thin_film_thickness=0.7, thin_film_ior=2.0)),
    ("thin film on a base without specular", dict(base_color=(0.5, 0.5, 0.5), specular_weight=0.0,
                                                  specular_roughness=0.2, thin_film_weight=1.0,
                                                  thin_film_thickness=0.5, thin_film_ior=1.5)),
    ("fuzz over plastic", dict(base_color=(0.6, 0.2, 0.2), specular_roughness=0.4, fuzz_weight=0.8,
                               fuzz_color=(0.9, 0.9, 1.0), fuzz_roughness=0.5)),
    ("fuzz over a delta coat on metal", dict(base_metalness=1.0, base_color=(0.8, 0.7, 0.4), specular_roughness=0.3,
                                             coat_weight=1.0, coat_roughness=0.0, fuzz_weight=0.5,
                                             fuzz_color=(1.0, 0.6, 0.8), fuzz_roughness=0.9)),
    ("fuzz over a smooth dielectric", dict(base_color=(0.2, 0.4, 0.2), specular_roughness=0.0, fuzz_weight=1.0,
                                           fuzz_color=(0.7, 0.8, 0.6), fuzz_roughness=0.2)),
]


def material_zoo(width=96, height=96, spp=8, max_depth=6, seed=0, sphere_level=2) -> Scene:
    """An open-topped box (floor, back, left and right walls, Lambert) under
    a small sky with a sun, a 0.3 x 0.3 quad light of radiance 12 hung below
    the open top, and fifteen icospheres (radius 0.085, level 2) in three
    rows, each with one of ZOO_MATERIALS: partial metalness, coat over metal,
    transmission over diffuse and over partial metal, tints of the
    specular, coat and transmission colours, specular_weight < 1,
    anisotropy under a coat, thin films, fuzz and subsurface — the OpenPBR
    mixes that the closed-box, icosphere-field and instanced scenes do not
    reach.  The back wall is a rough diffuse (base_diffuse_roughness 0.7),
    the left wall a rough diffuse base (0.3) under a glossy specular layer,
    the right wall a diffuse base with 40 % subsurface."""
    mats = [lambert((0.6, 0.6, 0.6)),
            material(base_color=(0.7, 0.4, 0.3), base_diffuse_roughness=0.7, specular_weight=0.0),
            material(base_color=(0.3, 0.6, 0.4), base_diffuse_roughness=0.3, specular_roughness=0.5),
            material(base_color=(0.4, 0.4, 0.7), specular_weight=0.0, subsurface_weight=0.4,
                     subsurface_color=(0.8, 0.6, 0.4)),
            material(base_weight=0.0, specular_weight=0.0, emission_luminance=12.0,
                     emission_color=(1.0, 0.95, 0.9))]
    mats += [material(**kw) for _, kw in ZOO_MATERIALS]
    b = _MeshBuilder()
    b.add_quad([0, 0, 0], [1, 0, 0], [1, 0, 1], [0, 0, 1], [0, 1, 0], 0)    # floor
    b.add_quad([0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1], [0, 0, -1], 1)   # back
    b.add_quad([0, 0, 0], [0, 1, 0], [0, 1, 1], [0, 0, 1], [1, 0, 0], 2)    # left
    b.add_quad([1, 0, 0], [1, 1, 0], [1, 1, 1], [1, 0, 1], [-1, 0, 0], 3)   # right
    b.add_quad([.35, .92, .45], [.65, .92, .45], [.65, .92, .75], [.35, .92, .75], [0, -1, 0], 4)
    v, f = icosphere(sphere_level)
    rad = 0.085
    for k in range(len(ZOO_MATERIALS)):
        row = k // 5
        cx = 0.14 + 0.18 * (k % 5)
        cz = (0.3, 0.58, 0.86)[row]
        cy = rad + (0.0, 0.13, 0.26)[row]
        b.add(v * rad + np.array([cx, cy, cz]), f, 5 + k)
    cam = Camera((0.5, 0.5, -0.45), (0.5, 0.18, 0.5), (0.0, 1.0, 0.0), 42.0, width, height)
    env = sky_env(width=256, height=128, sun_elev_deg=55.0, sun_azim_deg=160.0, sun_diam_deg=3.0,
                  sun_radiance=200.0)
    return Scene("material_zoo", [b.mesh()], [], np.stack(mats), env, cam, spp, max_depth, seed)


# --------------------------------------------------------------------------
# icosphere field (~1.31M triangles)
# --------------------------------------------------------------------------

def icosphere(level: int):
    """Unit icosphere: 20*4^level triangles, 10*4^level+2 vertices (float64)."""
    t = (1.0 + 5 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = v[uniq[:, 0]] + v[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = v.shape[0]
        v = np.concatenate([v, mid])
        nf = f.shape[0]
        a = base + inv[:nf]
        b_ = base + inv[nf:2 * nf]
        c = base + inv[2 * nf:]
        f = np.concatenate([
            np.stack([f[:, 0], a, c], 1), np.stack([f[:, 1], b_, a], 1),
            np.stack([f[:, 2], c, b_], 1), np.stack([a, b_, c], 1)])
    return v, f


class ValueNoise:
    """Trilinear value noise on the integer lattice, smoothstep-weighted.

    Lattice value at (i,j,k) is vals[perm[(perm[(perm[i&255]+j)&255]+k)&255]]
    with a seeded permutation `perm` and lattice values U[0,1).
    Output is in [0,1).
    """

    def __init__(self, seed: int):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.perm = rng.permutation(256).astype(np.int64)
        self.vals = rng.uniform(0.0, 1.0, 256)

    def _lat(self, i, j, k):
        p = self.perm
        return self.vals[p[(p[(p[i & 255] + j) & 255] + k) & 255]]

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        fl = np.floor(x)
        i = fl.astype(np.int64)
        f = x - fl
        w = f * f * (3.0 - 2.0 * f)
        out = 0.0
        for dx in (0, 1):
            wx = w[:, 0] if dx else 1.0 - w[:, 0]
            for dy in (0, 1):
                wy = w[:, 1] if dy else 1.0 - w[:, 1]
                for dz in (0, 1):
                    wz = w[:, 2] if dz else 1.0 - w[:, 2]
                    out = out + wx * wy * wz * self._lat(i[:, 0] + dx, i[:, 1] + dy, i[:, 2] + dz)
        return out


def sky_env(width=2048, height=1024, sun_elev_deg=35.0, sun_azim_deg=135.0,
            sun_diam_deg=0.5, sun_radiance=1e4, sub=16) -> np.ndarray:
    """Equirect (y up) sky: for d_y >= 0 sky = H + (Z-H)*sqrt(d_y) with
    H=(.85,.9,1), Z=(.25,.45,.95); below the horizon (.12,.11,.10).  A disc
    sun of the given angular diameter and radiance is added; each texel near
    it gets sun_radiance x (fraction of sub x sub sub-samples inside the
    disc).  Texel (row r, col c) centre: u=(c+.5)/W, v=(r+.5)/H,
    theta = pi v, phi = 2 pi (u - 1/2), d = (sin t sin p, cos t, -sin t cos p).
    """
    H = np.array([0.85, 0.90, 1.00])
    Z = np.array([0.25, 0.45, 0.95])
    G = np.array([0.12, 0.11, 0.10])
    v = (np.arange(height) + 0.5) / height
    th = np.pi * v
    dy = np.cos(th)
    row = np.where(dy[:, None] >= 0, H + (Z - H) * np.sqrt(np.maximum(dy, 0.0))[:, None], G)
    env = np.broadcast_to(row[:, None, :], (height, width, 3)).astype(np.float64).copy()
    # sun direction in the same parametrisation
    st = math.radians(90.0 - sun_elev_deg)
    sp = math.radians(sun_azim_deg)
    s = np.array([math.sin(st) * math.sin(sp), math.cos(st), -math.sin(st) * math.cos(sp)])
    cos_r = math.cos(math.radians(sun_diam_deg / 2.0))
    # texel window around the sun
    r0 = max(0, int(math.floor((st - 0.02) / math.pi * height)))
    r1 = min(height, int(math.ceil((st + 0.02) / math.pi * height)) + 1)
    for r in range(r0, r1):
        for c in range(width):
            uc = (c + 0.5) / width
            phi = 2 * math.pi * (uc - 0.5)
            thc = math.pi * (r + 0.5) / height
            dc = np.array([math.sin(thc) * math.sin(phi), math.cos(thc), -math.sin(thc) * math.cos(phi)])
            if dc @ s < math.cos(math.radians(2.0)):
                continue
            uu = (c + (np.arange(sub) + 0.5) / sub) / width
            vv = (r + (np.arange(sub) + 0.5) / sub) / height
            T, P = np.meshgrid(np.pi * vv, 2 * np.pi * (uu - 0.5), indexing="ij")
            d = np.stack([np.sin(T) * np.sin(P), np.cos(T), -np.sin(T) * np.cos(P)], -1)
            frac = float(np.mean((d @ s) >= cos_r))
            env[r, c] += sun_radiance * frac
    return env.astype(np.float32)


def spheres(width=1920, height=1080, spp=64, max_depth=8, seed=0, level=5,
            env_size=(2048, 1024)) -> Scene:
    """64 icospheres (level 5 -> 20,480 tris each) radially displaced by
    r = 1 + 0.15 n(v), n = sum_{o=0..2} 0.5^o N(2^o * 2 v + off_i) / 1.75,
    on an 8x8 grid of pitch 3 with centres at y = 1.2, plus a 2-triangle
    ground [-50,50]^2 at y = 0: 1,310,722 triangles at level 5.

    Per sphere (PCG64(2) draws, sphere order row-major over the grid):
    off_i ~ U[0,100)^3; Bernoulli(1/2) picks metal (metalness 1, base_color
    U[.5,.95]^3, specular_roughness U[.05,.6]) or coated diffuse (base_color
    U[.2,.8]^3, specular_roughness 0.3, ior 1.5, coat_weight 1, coat_ior 1.5,
    coat_roughness 0).  Ground: Lambert 0.5.  Lighting: sky_env().
    """
    rng = np.random.Generator(np.random.PCG64(2))
    noise = ValueNoise(1)
    uv, uf = icosphere(level)
    mats = [lambert((0.5, 0.5, 0.5))]
    b = _MeshBuilder()
    b.add_quad([-50, 0, -50], [50, 0, -50], [50, 0, 50], [-50, 0, 50], [0, 1, 0], 0)
    for gz in range(8):
        for gx in range(8):
            off = rng.uniform(0.0, 100.0, 3)
            n = np.zeros(uv.shape[0])
            for o in range(3):
                n += 0.5 ** o * noise((2.0 ** o) * 2.0 * uv + off)
            n /= 1.75
            r = 1.0 + 0.15 * n
            centre = np.array([-10.5 + 3.0 * gx, 1.2, -10.5 + 3.0 * gz])
            verts = uv * r[:, None] + centre
            if rng.uniform() < 0.5:
                col = rng.uniform(0.5, 0.95, 3)
                rough = rng.uniform(0.05, 0.6)
                mats.append(material(base_color=tuple(col), base_metalness=1.0,
                                     specular_roughness=float(rough)))
            else:
                col = rng.uniform(0.2, 0.8, 3)
                mats.append(material(base_color=tuple(col), specular_roughness=0.3,
                                     specular_ior=1.5, coat_weight=1.0, coat_ior=1.5,
                                     coat_roughness=0.0))
            b.add(verts, uf, len(mats) - 1)
    env = sky_env(*env_size)
    cam = Camera((0.0, 9.0, 22.0), (0.0, 0.5, 0.0), (0.0, 1.0, 0.0), 40.0, width, height)
    return Scene("spheres", [b.mesh()], [], np.stack(mats), env, cam, spp, max_depth, seed)


# --------------------------------------------------------------------------
# instanced CAD-like scene (~10.8M instanced triangles)
# --------------------------------------------------------------------------

def lathe(profile, n_seg: int, closed_loop: bool = False):
    """Closed surface of revolution about +y from a 2-D profile [(r, y), ...].

    An open profile must start and end on the axis (r = 0): those ends become
    triangle fans.  A closed loop (e.g. a torus section) wraps around.  Rings
    share vertices around the seam, so the mesh is watertight.  Triangles are
    wound with outward normals for a counter-clockwise profile (r increasing
    along the bottom).
    """
    prof = np.asarray(profile, dtype=np.float64)
    ang = 2.0 * np.pi * np.arange(n_seg) / n_seg
    ca, sa = np.cos(ang), np.sin(ang)
    verts, rings = [], []
    for (r, y) in prof:
        if r == 0.0 and not closed_loop:
            rings.append([len(verts)] * n_seg)
            verts.append((0.0, y, 0.0))
        else:
            base = len(verts)
            verts.extend(zip(r * ca, np.full(n_seg, y), r * sa))
            rings.append(list(range(base, base + n_seg)))
    tris = []
    n_rings = len(rings)
    last = n_rings if closed_loop else n_rings - 1
    for i in range(last):
        a, b = rings[i], rings[(i + 1) % n_rings]
        for j in range(n_seg):
            j1 = (j + 1) % n_seg
            q = (a[j], a[j1], b[j1], b[j])
            tri1, tri2 = (q[0], q[2], q[1]), (q[0], q[3], q[2])
            for t in (tri1, tri2):
                if len({t[0], t[1], t[2]}) == 3:
                    tris.append(t)
    return np.asarray(verts, dtype=np.float64), np.asarray(tris, dtype=np.int64)


def _arc(cx, cy, rad, a0, a1, n):
    t = np.linspace(a0, a1, n)
    return [(cx + rad * np.cos(x), cy + rad * np.sin(x)) for x in t]


def bevelled_cylinder(radius, height, bevel, n_seg, n_bevel, n_side):
    """Cylinder with rounded (bevelled) rims, closed by flat caps."""
    h = height / 2.0
    prof = [(0.0, -h)]
    prof += [(x, -h) for x in np.linspace(0.0, radius - bevel, 4)[1:]]
    prof += _arc(radius - bevel, -h + bevel, bevel, -np.pi / 2, 0.0, n_bevel)[1:]
    prof += [(radius, y) for y in np.linspace(-h + bevel, h - bevel, n_side)[1:-1]]
    prof += _arc(radius - bevel, h - bevel, bevel, 0.0, np.pi / 2, n_bevel)
    prof += [(x, h) for x in np.linspace(radius - bevel, 0.0, 4)[1:]]
    return lathe(prof, n_seg)


def torus(R, r, n_seg, n_ring):
    prof = [(R + r * np.cos(a), r * np.sin(a)) for a in 2 * np.pi * np.arange(n_ring) / n_ring]
    return lathe(prof, n_seg, closed_loop=True)


def _quat_to_matrix(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _shoemake(u1, u2, u3):
    """Uniform random rotation from three uniforms (Shoemake, Graphics Gems III)."""
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    return _quat_to_matrix((b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                            a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)))


def instanced(width=1920, height=1080, spp=256, max_depth=12, seed=0, env_size=(2048, 1024)) -> Scene:
    """400 instances of 5 closed lathe meshes (bevelled cylinders and tori of
    about 10k, 17.5k, 25k, 32.5k and 50k triangles, bounding radius <= 1.3)
    on a jittered 20x20 grid of pitch 2.8, each lifted to y = radius + U[0,2]
    and rotated uniformly at random: ~10.8M instanced triangles.  A ground
    plane and four 2x2 quad lights (radiance 20, at y = 12 above (+-8, +-8))
    are identity instances.

    Materials per instance, labels shuffled 120 / 160 / 120 (PCG64(3) draws):
    glass (transmission 1, IOR 1.5, roughness 0.02), brushed metal
    (metalness 1, roughness 0.3, anisotropy 0.7, base_color U[.6,.95]^3),
    coated plastic (base_color U[.1,.9]^3, roughness 0.4, coat 1 at IOR 1.5,
    coat roughness 0.05).  Lighting: the sky of spheres() plus the quads.
    """
    rng = np.random.Generator(np.random.PCG64(3))
    objs = [torus(0.9, 0.35, 100, 50),
            bevelled_cylinder(0.8, 1.6, 0.12, 175, 12, 24),
            torus(0.85, 0.4, 125, 100),
            bevelled_cylinder(0.75, 1.8, 0.2, 250, 18, 27),
            torus(0.9, 0.38, 200, 125)]
    meshes = []
    radius = []
    for v, f in objs:
        c = 0.5 * (v.min(0) + v.max(0))
        v = v - c
        radius.append(float(np.linalg.norm(v, axis=1).max()))
        meshes.append(Mesh(v.astype(np.float32), f.astype(np.int32), np.zeros(len(f), np.int32)))
    assert max(radius) <= 1.3
    labels = np.array([0] * 120 + [1] * 160 + [2] * 120)
    rng.shuffle(labels)
    mats, insts = [], []
    for k in range(400):
        gx, gz = k % 20, k // 20
        mesh_id = int(rng.integers(0, 5))
        jit = rng.uniform(-0.1, 0.1, 2)
        x = -26.6 + 2.8 * gx + jit[0]
        z = -26.6 + 2.8 * gz + jit[1]
        y = radius[mesh_id] + rng.uniform(0.0, 2.0)
        R = _shoemake(*rng.uniform(size=3))
        M = np.zeros((3, 4))
        M[:, :3] = R
        M[:, 3] = (x, y, z)
        lab = labels[k]
        if lab == 0:
            mats.append(material(base_weight=0.0, transmission_weight=1.0, specular_ior=1.5,
                                 specular_roughness=0.02))
        elif lab == 1:
            mats.append(material(base_color=tuple(rng.uniform(0.6, 0.95, 3)), base_metalness=1.0,
                                 specular_roughness=0.3, specular_roughness_anisotropy=0.7))
        else:
            mats.append(material(base_color=tuple(rng.uniform(0.1, 0.9, 3)), specular_roughness=0.4,
                                 coat_weight=1.0, coat_ior=1.5, coat_roughness=0.05))
        insts.append(Instance(M.astype(np.float32), mesh_id, len(mats) - 1))
    # ground (identity instance)
    g = _MeshBuilder()
    g.add_quad([-50, 0, -50], [50, 0, -50], [50, 0, 50], [-50, 0, 50], [0, 1, 0], 0)
    meshes.append(g.mesh())
    mats.append(lambert((0.5, 0.5, 0.5)))
    eye = np.hstack([np.eye(3), np.zeros((3, 1))]).astype(np.float32)
    insts.append(Instance(eye, 5, len(mats) - 1))
    # four quad lights facing down (identity instance)
    lq = _MeshBuilder()
    for cx in (-8.0, 8.0):
        for cz in (-8.0, 8.0):
            lq.add_quad([cx - 1, 12, cz - 1], [cx + 1, 12, cz - 1], [cx + 1, 12, cz + 1], [cx - 1, 12, cz + 1],
                        [0, -1, 0], 0)
    meshes.append(lq.mesh())
    mats.append(material(base_weight=0.0, specular_weight=0.0, emission_luminance=20.0))
    insts.append(Instance(eye, 6, len(mats) - 1))
    env = sky_env(*env_size)
    cam = Camera((0.0, 14.0, 34.0), (0.0, 1.0, 0.0), (0.0, 1.0, 0.0), 40.0, width, height)
    return Scene("instanced", meshes, insts, np.stack(mats), env, cam, spp, max_depth, seed)


# --------------------------------------------------------------------------
# test scenes with closed-form answers
# --------------------------------------------------------------------------

def uniform_env(value=1.0, width=64, height=32, upper_only=False) -> np.ndarray:
    env = np.full((height, width, 3), value, dtype=np.float32)
    if upper_only:
        v = (np.arange(height) + 0.5) / height
        env[np.cos(np.pi * v) < 0] = 0.0
    return env


def furnace(kind="sphere", width=32, height=32, spp=8, max_depth=256, seed=0,
            mat=None, level=2) -> Scene:
    """An object under a uniform environment of radiance 1.

    kind: "sphere" (icosphere, convex), "cubes" (the two box-scene cubes on a
    floor quad, not convex), "glass" (smooth dielectric icosphere, IOR 1.5).
    Default material: white Lambert (albedo 1).
    """
    b = _MeshBuilder()
    if mat is None:
        mat = lambert((1.0, 1.0, 1.0))
    if kind == "glass":
        mat = material(base_weight=0.0, specular_roughness=0.0, specular_ior=1.5,
                       transmission_weight=1.0)
    if kind in ("sphere", "glass"):
        v, f = icosphere(level)
        b.add(v * 0.5 + np.array([0.5, 0.5, 0.5]), f, 0)
    elif kind == "cubes":
        b.add_quad([-.5, 0, -.5], [1.5, 0, -.5], [1.5, 0, 1.5], [-.5, 0, 1.5], [0, 1, 0], 0)
        for f_ in _box_faces([.15, 0, .15], [.45, .30, .45]):
            b.add_quad(*f_, 0)
        for f_ in _box_faces([.55, 0, .50], [.85, .60, .80]):
            b.add_quad(*f_, 0)
    else:
        raise ValueError(kind)
    cam = Camera((0.5, 0.5, -1.4), (0.5, 0.5, 0.0), (0.0, 1.0, 0.0), 40.0, width, height)
    return Scene("furnace_" + kind, [b.mesh()], [], np.stack([mat]), uniform_env(1.0),
                 cam, spp, max_depth, seed)


def plane(rho=(0.3, 0.5, 0.7), L=2.0, width=32, height=32, spp=8, max_depth=4, seed=0) -> Scene:
    """A Lambert plane of albedo rho (y = 0, 2 triangles over [-1e3,1e3]^2)
    under a sky of radiance L for d_y > 0 and 0 below.  Plane pixels converge
    to rho*L, sky pixels are L."""
    b = _MeshBuilder()
    s = 1000.0
    b.add_quad([-s, 0, -s], [s, 0, -s], [s, 0, s], [-s, 0, s], [0, 1, 0], 0)
    cam = Camera((0.0, 1.0, 0.0), (0.0, 0.6, -2.0), (0.0, 1.0, 0.0), 60.0, width, height)
    return Scene("plane", [b.mesh()], [], np.stack([lambert(rho)]),
                 uniform_env(L, upper_only=True), cam, spp, max_depth, seed)


def display_sums(width=1920, height=1080, samples=64, seed=0) -> np.ndarray:
    """Seeded FP64 per-pixel sums [height, width, 3] of `samples` samples for
    the display path: mean radiance log-uniform over [1e-4, 1e3] per pixel,
    with colour ratios U[0.05, 1] per channel, plus rows of special values
    (black, exact greys from 0 to 20, the values 0.08 and 0.76 + 0.04 in
    every channel, one dark channel, and a ramp of greys that steps across
    8-bit code boundaries).  Data only; no display arithmetic."""
    r = np.random.Generator(np.random.PCG64(seed))
    mag = 10.0 ** r.uniform(-4.0, 3.0, size=(height, width, 1))
    mean = mag * r.uniform(0.05, 1.0, size=(height, width, 3))
    specials = [np.zeros(3), np.full(3, 0.08), np.full(3, 0.8), np.array([0.0, 0.5, 2.0]),
                np.array([0.079, 0.3, 0.9]), np.array([1e-9, 1e-9, 1e-9]), np.array([50.0, 0.1, 0.1])]
    k = 0
    for y in range(min(height, 4)):
        for x in range(width):
            if k < len(specials):
                mean[y, x] = specials[k]
            else:
                mean[y, x] = np.full(3, 20.0 * (k - len(specials)) / max(1, 4 * width - len(specials)))
            k += 1
    return mean * float(samples)
