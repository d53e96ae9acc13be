"""ctypes wrapper of the FP64 oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Scenes are duck-typed (attributes meshes, instances, materials, env,
camera), so this module does not import the HIP package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            import importlib.util
            spec = importlib.util.spec_from_file_location("_oracle_build", os.path.join(HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class OMesh(C.Structure):
    _fields_ = [("vertices", C.c_void_p), ("n_vertices", C.c_int64), ("indices", C.c_void_p),
                ("n_triangles", C.c_int64), ("material_ids", C.c_void_p)]


class OInstance(C.Structure):
    _fields_ = [("object_to_world", C.c_float * 12), ("mesh", C.c_int32), ("material_override", C.c_int32)]


class OCamera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class OOptions(C.Structure):
    _fields_ = [("estimator", C.c_int32), ("russian_roulette", C.c_int32), ("n_threads", C.c_int32),
                ("verbose", C.c_int32), ("nrc_weights", C.c_void_p), ("nrc_bounce", C.c_int32),
                ("nrc_bf16", C.c_int32), ("train_end", C.c_int32), ("nrc_factor", C.c_int32),
                ("spread_c", C.c_double)]


class OStats(C.Structure):
    _fields_ = [("extension_rays", C.c_int64), ("shadow_rays", C.c_int64), ("dropped_nonfinite", C.c_int64)]


MIS, BSDF_ONLY, NEE_ONLY = 0, 1, 2

_dp = C.POINTER(C.c_double)


def _declare(L):
    L.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    L.oracle_philox4x32_10.restype = None
    L.oracle_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
    L.oracle_uniform.restype = C.c_double
    L.oracle_scene_create.argtypes = [C.POINTER(OMesh), C.c_int32, C.POINTER(OInstance), C.c_int32,
                                      C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_void_p)]
    L.oracle_scene_destroy.argtypes = [C.c_void_p]
    L.oracle_scene_destroy.restype = None
    L.oracle_scene_tmin.argtypes = [C.c_void_p]
    L.oracle_scene_tmin.restype = C.c_double
    L.oracle_scene_n_lights.argtypes = [C.c_void_p]
    L.oracle_scene_n_lights.restype = C.c_int64
    L.oracle_camera_ray.argtypes = [C.POINTER(OCamera), C.c_double, C.c_double, _dp, _dp]
    for name in ("oracle_closest_f64", "oracle_closest_f64_brute"):
        f = getattr(L, name)
        f.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_int32, C.c_int32, _dp,
                      C.POINTER(C.c_int32)]
    L.oracle_closest_f32_brute.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32]
    L.oracle_trace_path.argtypes = [C.c_void_p, C.POINTER(OCamera), C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int32, C.c_uint64, C.POINTER(OOptions), _dp,
                                    C.POINTER(C.c_uint64), C.POINTER(OStats)]
    L.oracle_render.argtypes = [C.c_void_p, C.POINTER(OCamera), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(OOptions),
                                C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(OStats)]
    L.oracle_bsdf_eval.argtypes = [C.c_void_p, C.c_int32, _dp, _dp, _dp, _dp]
    L.oracle_bsdf_sample.argtypes = [C.c_void_p, C.c_int32, _dp, _dp, _dp, _dp, _dp,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.oracle_lobe_pmf.argtypes = [C.c_void_p, C.c_int32, C.c_double, _dp]
    L.oracle_lobe_pmf.restype = None
    L.oracle_fresnel_dielectric.argtypes = [C.c_double, C.c_double]
    L.oracle_fresnel_dielectric.restype = C.c_double
    L.oracle_fuzz_albedo.argtypes = [C.c_double, C.c_double]
    L.oracle_fuzz_albedo.restype = C.c_double
    L.oracle_film_reflectance.argtypes = [C.c_double] * 6
    L.oracle_film_reflectance.restype = C.c_double
    L.oracle_fresnel_f82.argtypes = [C.c_void_p, C.c_double, _dp]
    L.oracle_fresnel_f82.restype = None
    L.oracle_ggx_D.argtypes = [C.c_double, C.c_double, _dp]
    L.oracle_ggx_D.restype = C.c_double
    L.oracle_ggx_G1.argtypes = [C.c_double, C.c_double, _dp]
    L.oracle_ggx_G1.restype = C.c_double
    L.oracle_ggx_vndf_sample.argtypes = [C.c_double, C.c_double, _dp, C.c_double, C.c_double, _dp]
    L.oracle_ggx_vndf_sample.restype = None
    L.oracle_ggx_vndf_pdf.argtypes = [C.c_double, C.c_double, _dp, _dp]
    L.oracle_ggx_vndf_pdf.restype = C.c_double
    L.oracle_sample_light.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp,
                                      _dp, C.POINTER(C.c_int64)]
    L.oracle_env_pdf.argtypes = [C.c_void_p, _dp]
    L.oracle_env_pdf.restype = C.c_double
    L.oracle_env_radiance.argtypes = [C.c_void_p, _dp, _dp]
    L.oracle_env_radiance.restype = None
    L.oracle_bf16_round.argtypes = [C.c_double]
    L.oracle_bf16_round.restype = C.c_double
    L.oracle_nrc_encode.argtypes = [_dp, _dp]
    L.oracle_nrc_encode.restype = None
    L.oracle_nrc_forward.argtypes = [_dp, _dp, C.c_int32, _dp]
    L.oracle_nrc_forward.restype = None
    L.oracle_nrc_inputs.argtypes = [_dp, _dp, _dp, _dp, _dp, C.c_void_p, _dp]
    L.oracle_nrc_inputs.restype = None
    L.oracle_shading_frame.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.oracle_shading_frame.restype = None
    L.oracle_pbr_neutral.argtypes = [_dp, _dp]
    L.oracle_pbr_neutral.restype = None
    L.oracle_srgb_encode.argtypes = [C.c_double]
    L.oracle_srgb_encode.restype = C.c_double
    L.oracle_display.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_void_p, C.c_void_p]
    L.oracle_display.restype = None
    L.oracle_training_records.argtypes = [C.c_void_p, C.POINTER(OCamera), C.c_int32, C.c_int32, C.c_int32,
                                          C.c_int32, C.c_uint64, C.c_void_p, _dp, _dp, C.POINTER(C.c_int32)]


def _d3(x):
    return (C.c_double * 3)(*[float(v) for v in x])


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


# ------------------------------------------------------------ primitives --

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def uniform(seed, pixel, sample, bounce, dim):
    return lib().oracle_uniform(seed, pixel, sample, bounce, dim)


def camera_struct(cam) -> OCamera:
    c = OCamera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.look_at[:] = [float(x) for x in cam.look_at]
    c.up[:] = [float(x) for x in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


def camera_ray(cam, fx, fy):
    o = (C.c_double * 3)()
    d = (C.c_double * 3)()
    rc = lib().oracle_camera_ray(C.byref(camera_struct(cam)), fx, fy, o, d)
    assert rc == 0
    return np.array(o[:]), np.array(d[:])


def _mat(m) -> np.ndarray:
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(39))
    return m


def bsdf_eval(mat, wo, wi, entering=1):
    m = _mat(mat)
    f = (C.c_double * 3)()
    pdf = C.c_double()
    lib().oracle_bsdf_eval(m.ctypes.data, entering, _d3(wo), _d3(wi), f, C.byref(pdf))
    return np.array(f[:]), pdf.value


def bsdf_sample(mat, wo, u, entering=1):
    m = _mat(mat)
    uu = (C.c_double * 4)(*[float(x) for x in u])
    wi = (C.c_double * 3)()
    w = (C.c_double * 3)()
    pdf = C.c_double()
    flags = C.c_int32()
    lobe = C.c_int32()
    ok = lib().oracle_bsdf_sample(m.ctypes.data, entering, _d3(wo), uu, wi, w, C.byref(pdf),
                                  C.byref(flags), C.byref(lobe))
    return dict(ok=bool(ok), wi=np.array(wi[:]), weight=np.array(w[:]), pdf=pdf.value,
                delta=bool(flags.value & 1), refract=bool(flags.value & 2), lobe=lobe.value)


def lobe_pmf(mat, mu_o, entering=1):
    m = _mat(mat)
    p = (C.c_double * 5)()
    lib().oracle_lobe_pmf(m.ctypes.data, entering, mu_o, p)
    return np.array(p[:])


def fresnel_dielectric(c, eta):
    return lib().oracle_fresnel_dielectric(c, eta)


def fuzz_albedo(rough, mu):
    """Directional albedo of the fuzz lobe (weight 1, colour 1) from the oracle's table."""
    return lib().oracle_fuzz_albedo(rough, mu)


def film_reflectance(c, n2, n3, film_ior, d_nm, lambda_nm):
    """Unpolarised reflectance of a thin film (relative index n2) on a base (relative index n3)."""
    return lib().oracle_film_reflectance(c, n2, n3, film_ior, d_nm, lambda_nm)


def fresnel_f82(mat, mu):
    m = _mat(mat)
    F = (C.c_double * 3)()
    lib().oracle_fresnel_f82(m.ctypes.data, mu, F)
    return np.array(F[:])


def bf16_round(x):
    return lib().oracle_bf16_round(float(x))


def nrc_encode(x12):
    f = (C.c_double * 64)()
    lib().oracle_nrc_encode((C.c_double * 12)(*[float(v) for v in x12]), f)
    return np.array(f[:])


def nrc_forward(W, x12, bf16=False):
    w = np.ascontiguousarray(W, dtype=np.float64)
    y = (C.c_double * 3)()
    lib().oracle_nrc_forward(w.ctypes.data_as(_dp), (C.c_double * 12)(*[float(v) for v in x12]), 1 if bf16 else 0, y)
    return np.array(y[:])


def nrc_inputs(lo, hi, p, wo, n, mat):
    """The 12 cache inputs at point p of a scene box [lo, hi] (test hook)."""
    m = _mat(mat)
    x = (C.c_double * 12)()
    lib().oracle_nrc_inputs(_d3(lo), _d3(hi), _d3(p), _d3(wo), _d3(n), m.ctypes.data, x)
    return np.array(x[:])


def shading_frame(n, object_to_world=None):
    """(t, b) of the shading frame at unit normal n (test hook)."""
    t = (C.c_double * 3)()
    b = (C.c_double * 3)()
    if object_to_world is None:
        lib().oracle_shading_frame(None, _d3(n), t, b)
    else:
        w = np.ascontiguousarray(np.asarray(object_to_world, dtype=np.float32).reshape(12))
        lib().oracle_shading_frame(w.ctypes.data, _d3(n), t, b)
    return np.array(t[:]), np.array(b[:])


def pbr_neutral(c):
    out = (C.c_double * 3)()
    lib().oracle_pbr_neutral(_d3(c), out)
    return np.array(out[:])


def srgb_encode(v):
    return lib().oracle_srgb_encode(float(v))


def display(sum_rgb, samples, exposure=1.0):
    """Display image of FP64 sums [h, w, 3]: (encoded [h, w, 3] in [0, 1], rgba8 [h, w, 4])."""
    s = np.ascontiguousarray(sum_rgb, dtype=np.float64)
    h, w = s.shape[:2]
    enc = np.zeros((h, w, 3))
    rgba = np.zeros((h, w, 4), np.uint8)
    lib().oracle_display(s.ctypes.data, h * w, 1.0 / samples, float(exposure), enc.ctypes.data, rgba.ctypes.data)
    return enc, rgba


def ggx_D(at, ab, m):
    return lib().oracle_ggx_D(at, ab, _d3(m))


def ggx_G1(at, ab, w):
    return lib().oracle_ggx_G1(at, ab, _d3(w))


def ggx_vndf_sample(at, ab, wo, u1, u2):
    m = (C.c_double * 3)()
    lib().oracle_ggx_vndf_sample(at, ab, _d3(wo), u1, u2, m)
    return np.array(m[:])


def ggx_vndf_pdf(at, ab, wo, m):
    return lib().oracle_ggx_vndf_pdf(at, ab, _d3(wo), _d3(m))


# ----------------------------------------------------------------- scene --

class OracleScene:
    """The oracle's own copy of a scene (its own BVH, lights and env CDFs)."""

    def __init__(self, scene):
        L = lib()
        self._keep = []
        meshes = (OMesh * len(scene.meshes))()
        for i, m in enumerate(scene.meshes):
            v = np.ascontiguousarray(m.vertices, dtype=np.float32)
            idx = np.ascontiguousarray(m.indices, dtype=np.int32)
            mid = np.ascontiguousarray(m.material_ids, dtype=np.int32)
            self._keep += [v, idx, mid]
            meshes[i].vertices = v.ctypes.data
            meshes[i].n_vertices = v.shape[0]
            meshes[i].indices = idx.ctypes.data
            meshes[i].n_triangles = idx.shape[0]
            meshes[i].material_ids = mid.ctypes.data
        n_inst = len(scene.instances)
        insts = (OInstance * max(1, n_inst))()
        for i, ins in enumerate(scene.instances):
            insts[i].object_to_world[:] = [float(x) for x in np.asarray(ins.object_to_world, np.float32).reshape(12)]
            insts[i].mesh = int(ins.mesh)
            insts[i].material_override = int(ins.material_override)
        mats = np.ascontiguousarray(scene.materials, dtype=np.float32)
        env = None if scene.env is None else np.ascontiguousarray(scene.env, dtype=np.float32)
        self._keep += [mats, env]
        h = C.c_void_p()
        rc = L.oracle_scene_create(meshes, len(scene.meshes), insts, n_inst, mats.ctypes.data,
                                   mats.shape[0], None if env is None else env.ctypes.data,
                                   0 if env is None else env.shape[1], 0 if env is None else env.shape[0],
                                   C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_scene_create failed ({rc})")
        self.h = h
        self.camera = scene.camera
        self._keep = [mats]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.oracle_scene_destroy(self.h)
        self.h = None

    @property
    def tmin(self):
        return lib().oracle_scene_tmin(self.h)

    @property
    def n_lights(self):
        return lib().oracle_scene_n_lights(self.h)

    def closest(self, o, d, tmin=None, tmax=np.inf, skip=(-1, -1), brute=False):
        hit = (C.c_double * 3)()
        ids = (C.c_int32 * 2)()
        f = lib().oracle_closest_f64_brute if brute else lib().oracle_closest_f64
        r = f(self.h, _d3(o), _d3(d), self.tmin if tmin is None else tmin, tmax, skip[0], skip[1], hit, ids)
        if r < 0:
            raise RuntimeError("oracle traversal failed")
        return (bool(r), hit[0], hit[1], hit[2], ids[0], ids[1])

    def closest_f32(self, rays: np.ndarray, n_threads=8) -> np.ndarray:
        """rays float32 [n,8] (o, tmin, d, tmax) -> uint32 [n,6] (t, inst, prim, b1, b2, hit)."""
        rays = np.ascontiguousarray(rays, dtype=np.float32)
        n = rays.shape[0]
        hits = np.zeros((n, 6), dtype=np.uint32)
        rc = lib().oracle_closest_f32_brute(self.h, rays.ctypes.data, n, hits.ctypes.data, n_threads)
        assert rc == 0
        return hits

    def trace_path(self, px, py, sample, max_depth, seed=0, estimator=MIS, rr=True, camera=None, verbose=False,
                   nrc_weights=None, nrc_bounce=2, nrc_bf16=False):
        cam = camera_struct(camera or self.camera)
        w = None if nrc_weights is None else np.ascontiguousarray(nrc_weights, dtype=np.float64)
        opt = OOptions(estimator, 1 if rr else 0, 1, 1 if verbose else 0, None if w is None else w.ctypes.data,
                       nrc_bounce, 1 if nrc_bf16 else 0, -1, 0)
        rgb = (C.c_double * 3)()
        sig = C.c_uint64()
        st = OStats()
        rc = lib().oracle_trace_path(self.h, C.byref(cam), px, py, sample, max_depth, seed, C.byref(opt),
                                     rgb, C.byref(sig), C.byref(st))
        if rc != 0:
            raise RuntimeError(f"oracle_trace_path failed ({rc})")
        return np.array(rgb[:]), int(sig.value)

    def render(self, spp, max_depth, seed=0, crop=None, first_sample=0, estimator=MIS, rr=True,
               per_sample=False, n_threads=None, camera=None, nrc_weights=None, nrc_bounce=2, nrc_bf16=False,
               nrc_factor=False, spread_c=0.0):
        """Returns dict(sum [h,w,3] f64, mean, per_sample [h,w,n,3], sigs [h,w,n] u64, stats)."""
        cam_py = camera or self.camera
        cam = camera_struct(cam_py)
        x0, y0, w, h = crop if crop is not None else (0, 0, cam_py.width, cam_py.height)
        nt = n_threads or min(16, os.cpu_count() or 1)
        wts = None if nrc_weights is None else np.ascontiguousarray(nrc_weights, dtype=np.float64)
        opt = OOptions(estimator, 1 if rr else 0, nt, 0, None if wts is None else wts.ctypes.data, nrc_bounce,
                       1 if nrc_bf16 else 0, -1, 1 if nrc_factor else 0, float(spread_c))
        s = np.zeros((h, w, 3), dtype=np.float64)
        ps = np.zeros((h, w, spp, 3), dtype=np.float64) if per_sample else None
        sg = np.zeros((h, w, spp), dtype=np.uint64) if per_sample else None
        st = OStats()
        rc = lib().oracle_render(self.h, C.byref(cam), x0, y0, w, h, first_sample, spp, max_depth, seed,
                                 C.byref(opt), s.ctypes.data, None if ps is None else ps.ctypes.data,
                                 None if sg is None else sg.ctypes.data, C.byref(st))
        if rc != 0:
            raise RuntimeError(f"oracle_render failed ({rc})")
        return dict(sum=s, mean=s / max(spp, 1), per_sample=ps, sigs=sg,
                    stats=dict(extension_rays=st.extension_rays, shadow_rays=st.shadow_rays,
                               dropped_nonfinite=st.dropped_nonfinite, threads=nt))

    def training_records(self, px, py, sample, max_depth, seed=0, camera=None, nrc_weights=None, train_end=-1,
                         nrc_bf16=False, factorize=False, rr=True):
        """Cache training records of one path: (inputs [k,12], targets [k,3]).  With weights and
        train_end >= 0 the path ends in the cache at that vertex (self-training)."""
        cam = camera_struct(camera or self.camera)
        x = np.zeros((max_depth + 1, 12))
        t = np.zeros((max_depth + 1, 3))
        n = C.c_int32()
        wts = None if nrc_weights is None else np.ascontiguousarray(nrc_weights, dtype=np.float64)
        opt = OOptions(MIS, 1 if rr else 0, 1, 0, None if wts is None else wts.ctypes.data, -1, 1 if nrc_bf16 else 0,
                       train_end if wts is not None else -1, 1 if factorize else 0)
        rc = lib().oracle_training_records(self.h, C.byref(cam), px, py, sample, max_depth, seed, C.byref(opt),
                                           _dptr(x), _dptr(t), C.byref(n))
        assert rc == 0
        return x[:n.value].copy(), t[:n.value].copy()

    def sample_light(self, p, usel, u1, u2):
        wl = (C.c_double * 3)()
        dist = C.c_double()
        pdf = C.c_double()
        Le = (C.c_double * 3)()
        lid = C.c_int64()
        ok = lib().oracle_sample_light(self.h, _d3(p), usel, u1, u2, wl, C.byref(dist), C.byref(pdf), Le,
                                       C.byref(lid))
        return dict(ok=bool(ok), wl=np.array(wl[:]), dist=dist.value, pdf=pdf.value, Le=np.array(Le[:]),
                    light=lid.value)

    def env_pdf(self, d):
        return lib().oracle_env_pdf(self.h, _d3(d))

    def env_radiance(self, d):
        Le = (C.c_double * 3)()
        lib().oracle_env_radiance(self.h, _d3(d), Le)
        return np.array(Le[:])
