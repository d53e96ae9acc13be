"""Thin ctypes binding of libpt.so (include/pt.h), same names as the C ABI.

Argument marshalling only: every step of the path runs in the HIP library.
Device buffers are torch tensors on the scene's GPU; their data pointers
cross the boundary.  If libpt.so is missing this module raises at import:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpt.so")

PT_OK = 0
STATUS = {0: "PT_OK", -1: "PT_ERR_INVALID_ARG", -2: "PT_ERR_OUT_OF_MEMORY", -3: "PT_ERR_DEVICE",
          -4: "PT_ERR_UNSUPPORTED", -5: "PT_ERR_STATE"}


class PtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class pt_mesh(C.Structure):
    _fields_ = [("vertices", C.c_void_p), ("n_vertices", C.c_int64), ("indices", C.c_void_p),
                ("n_triangles", C.c_int64), ("material_ids", C.c_void_p)]


class pt_instance(C.Structure):
    _fields_ = [("object_to_world", C.c_float * 12), ("mesh", C.c_int32), ("material_override", C.c_int32)]


class pt_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class pt_stats(C.Structure):
    _fields_ = [("extension_rays", C.c_int64), ("shadow_rays", C.c_int64), ("nonfinite_dropped", C.c_int64),
                ("samples", C.c_int64), ("ms_extend", C.c_double), ("launches_extend", C.c_int64),
                ("ms_total", C.c_double), ("node_visits", C.c_int64), ("tri_tests", C.c_int64),
                ("shadow_node_visits", C.c_int64), ("shadow_tri_tests", C.c_int64),
                ("cache_queries", C.c_int64), ("cache_records", C.c_int64), ("cache_adam_steps", C.c_int64),
                ("ms_cache_query", C.c_double), ("ms_cache_train", C.c_double),
                ("tail_extension_rays", C.c_int64), ("tail_node_visits", C.c_int64), ("tail_tri_tests", C.c_int64),
                ("ms_tail", C.c_double), ("launches_tail", C.c_int64),
                ("tail_shadow_rays", C.c_int64), ("tail_shadow_node_visits", C.c_int64),
                ("tail_shadow_tri_tests", C.c_int64), ("ms_display", C.c_double), ("launches_display", C.c_int64),
                ("instances_entered", C.c_int64), ("tail_instances_entered", C.c_int64),
                ("ms_cache_forward", C.c_double), ("cache_forward_queries", C.c_int64)]


class pt_bvh_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tris", C.c_int64), ("depth", C.c_int32),
                ("max_leaf_tris", C.c_int32), ("sah_cost", C.c_double), ("build_ms", C.c_double),
                ("stack_capacity", C.c_int32)]


class pt_radiance_cache_config(C.Structure):
    _fields_ = [("query_bounce", C.c_int32), ("train_paths", C.c_int32), ("batch_size", C.c_int32),
                ("steps_per_frame", C.c_int32), ("learning_rate", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("epsilon", C.c_float), ("init_seed", C.c_uint64), ("ema_decay", C.c_float),
                ("train_end_bounce", C.c_int32), ("spread_c", C.c_float), ("factorize", C.c_int32)]


NRC_PARAMS = 5 * 64 * 64 + 3 * 64


def cache_config(query_bounce=2, train_paths=1 << 16, batch_size=1 << 14, steps_per_frame=4, learning_rate=1e-3,
                 beta1=0.9, beta2=0.99, epsilon=1e-8, init_seed=0, ema_decay=0.0, train_end_bounce=-1,
                 spread_c=0.0, factorize=0):
    c = pt_radiance_cache_config()
    c.query_bounce, c.train_paths, c.batch_size, c.steps_per_frame = query_bounce, train_paths, batch_size, \
        steps_per_frame
    c.learning_rate, c.beta1, c.beta2, c.epsilon, c.init_seed = learning_rate, beta1, beta2, epsilon, init_seed
    c.ema_decay = ema_decay
    c.train_end_bounce, c.spread_c, c.factorize = train_end_bounce, spread_c, factorize
    return c


# every symbol declared in include/pt.h, with its ctypes signature
_SIGS = {
    "pt_scene_create": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pt_scene_destroy": (None, [C.c_void_p]),
    "pt_build_bvh": (C.c_int, [C.c_void_p, C.POINTER(pt_mesh), C.c_int32, C.POINTER(pt_instance), C.c_int32]),
    "pt_upload_materials": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "pt_set_environment": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "pt_render": (C.c_int, [C.c_void_p, C.POINTER(pt_camera), C.c_int32, C.c_int32, C.c_uint64, C.c_void_p]),
    "pt_accumulate": (C.c_int, [C.c_void_p, C.POINTER(pt_camera), C.c_int32, C.c_int32, C.c_int32, C.c_uint64]),
    "pt_reset_accumulation": (C.c_int, [C.c_void_p]),
    "pt_resolve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pt_render_debug": (C.c_int, [C.c_void_p, C.POINTER(pt_camera), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p]),
    "pt_trace_closest": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32]),
    "pt_trace_closest_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32]),
    "pt_display": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "pt_build_bvh_gpu": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "pt_set_gpu_bvh_builder": (C.c_int, [C.c_void_p, C.c_int32]),
    "pt_scene_bvh_info": (C.c_int, [C.c_void_p, C.POINTER(pt_bvh_info)]),
    "pt_scene_copy_bvh": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pt_set_accumulation": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64]),
    "pt_get_stats": (C.c_int, [C.c_void_p, C.POINTER(pt_stats)]),
    "pt_reset_stats": (C.c_int, [C.c_void_p]),
    "pt_set_profiling": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "pt_set_tail": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "pt_set_radiance_cache": (C.c_int, [C.c_void_p, C.POINTER(pt_radiance_cache_config)]),
    "pt_nrc_set_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "pt_nrc_get_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    "pt_nrc_get_inference_weights": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pt_nrc_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "pt_nrc_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                  C.POINTER(C.c_double)]),
    "pt_nrc_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_uint64,
                               C.POINTER(C.c_double)]),
    "pt_nrc_training_records": (C.c_int, [C.c_void_p, C.POINTER(pt_camera), C.c_int32, C.c_int32, C.c_uint64,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "pt_bvh_host_build": (C.c_int, [C.POINTER(pt_mesh), C.POINTER(C.c_void_p)]),
    "pt_bvh_host_build_instanced": (C.c_int, [C.POINTER(pt_mesh), C.c_int32, C.POINTER(pt_instance), C.c_int32,
                                              C.POINTER(C.c_void_p)]),
    "pt_bvh_host_info": (C.c_int, [C.c_void_p, C.POINTER(pt_bvh_info)]),
    "pt_bvh_host_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pt_bvh_host_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "pt_bvh_host_trace_stack": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                                          C.POINTER(C.c_int32)]),
    "pt_bvh_host_destroy": (None, [C.c_void_p]),
    "pt_last_error": (C.c_char_p, []),
    "pt_version": (C.c_char_p, []),
}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
# torch owns device memory and streams: load its HIP runtime first so that the
# library binds to the same runtime instead of bringing a second one.
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib():
    return _lib


def _check(status: int):
    if status != PT_OK:
        raise PtError(status, _lib.pt_last_error().decode())


def last_error() -> str:
    return _lib.pt_last_error().decode()


def version() -> str:
    return _lib.pt_version().decode()


def camera_struct(cam) -> pt_camera:
    c = pt_camera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.look_at[:] = [float(x) for x in cam.look_at]
    c.up[:] = [float(x) for x in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


def _mesh_structs(meshes, keep):
    arr = (pt_mesh * len(meshes))()
    for i, m in enumerate(meshes):
        v = np.ascontiguousarray(m.vertices, dtype=np.float32)
        idx = np.ascontiguousarray(m.indices, dtype=np.int32)
        mid = None if m.material_ids is None else np.ascontiguousarray(m.material_ids, dtype=np.int32)
        keep += [v, idx, mid]
        arr[i].vertices = v.ctypes.data
        arr[i].n_vertices = v.shape[0]
        arr[i].indices = idx.ctypes.data
        arr[i].n_triangles = idx.shape[0]
        arr[i].material_ids = None if mid is None else mid.ctypes.data
    return arr


class PtScene:
    """A pt_scene on one GPU.  Device buffers are torch tensors."""

    def __init__(self, device: int = 0, stream=None):
        import torch  # noqa: F401  (device memory and streams)
        self.device = device
        h = C.c_void_p()
        s = None if stream is None else C.c_void_p(stream)
        _check(_lib.pt_scene_create(device, s, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pt_scene_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()

    # -- set-up
    def build_bvh(self, meshes, instances=(), on_device=False):
        keep = []
        arr = _mesh_structs(meshes, keep)
        ni = len(instances)
        ia = (pt_instance * max(1, ni))()
        for i, ins in enumerate(instances):
            ia[i].object_to_world[:] = [float(x) for x in np.asarray(ins.object_to_world, np.float32).reshape(12)]
            ia[i].mesh = int(ins.mesh)
            ia[i].material_override = int(ins.material_override)
        build = _lib.pt_build_bvh_gpu if on_device else _lib.pt_build_bvh
        _check(build(self.h, arr, len(meshes), ia, ni))

    def set_gpu_bvh_builder(self, builder: str):
        """Builder of later build_bvh(on_device=True) calls: "ploc" (default) or "lbvh"."""
        _check(_lib.pt_set_gpu_bvh_builder(self.h, {"ploc": 0, "lbvh": 1}.get(builder, -1)))

    def bvh_info(self) -> dict:
        info = pt_bvh_info()
        _check(_lib.pt_scene_bvh_info(self.h, C.byref(info)))
        return {k: getattr(info, k) for k, _ in pt_bvh_info._fields_}

    def copy_bvh(self):
        """(nodes uint8 [n_nodes, 128], triangle records uint8 [n_tris, 48]) of the mesh-level BVH."""
        info = self.bvh_info()
        nodes = np.zeros((info["n_nodes"], 128), np.uint8)
        tris = np.zeros((info["n_tris"], 48), np.uint8)
        _check(_lib.pt_scene_copy_bvh(self.h, nodes.ctypes.data, tris.ctypes.data))
        return nodes, tris

    def upload_materials(self, materials: np.ndarray):
        m = np.ascontiguousarray(materials, dtype=np.float32).reshape(-1, 39)
        _check(_lib.pt_upload_materials(self.h, m.ctypes.data, m.shape[0]))

    def set_environment(self, env: Optional[np.ndarray]):
        if env is None:
            _check(_lib.pt_set_environment(self.h, None, 0, 0))
            return
        e = np.ascontiguousarray(env, dtype=np.float32)
        _check(_lib.pt_set_environment(self.h, e.ctypes.data, e.shape[1], e.shape[0]))

    # -- sampling
    def render(self, camera, spp, max_depth, seed, out):
        _check(_lib.pt_render(self.h, C.byref(camera_struct(camera)), spp, max_depth, seed, out.data_ptr()))
        return out

    def accumulate(self, camera, first_sample, n_samples, max_depth, seed):
        _check(_lib.pt_accumulate(self.h, C.byref(camera_struct(camera)), first_sample, n_samples, max_depth, seed))

    def reset_accumulation(self):
        _check(_lib.pt_reset_accumulation(self.h))

    def resolve(self, out, out_sum=None):
        _check(_lib.pt_resolve(self.h, out.data_ptr(), None if out_sum is None else out_sum.data_ptr()))
        return out

    def render_debug(self, camera, x0, y0, w, h, first_sample, spp, max_depth, seed, per_sample, sigs):
        _check(_lib.pt_render_debug(self.h, C.byref(camera_struct(camera)), x0, y0, w, h, first_sample, spp,
                                    max_depth, seed, per_sample.data_ptr(), sigs.data_ptr()))

    # -- radiance cache (device tensors: float32 on the scene's GPU)
    def set_radiance_cache(self, config=None):
        _check(_lib.pt_set_radiance_cache(self.h, None if config is None else C.byref(config)))

    def nrc_set_weights(self, w):
        _check(_lib.pt_nrc_set_weights(self.h, w.data_ptr(), w.numel()))

    def nrc_get_inference_weights(self, w):
        _check(_lib.pt_nrc_get_inference_weights(self.h, w.data_ptr()))
        return w

    def nrc_get_weights(self, w=None, m=None, v=None):
        step = C.c_int64(0)
        _check(_lib.pt_nrc_get_weights(self.h, None if w is None else w.data_ptr(),
                                       None if m is None else m.data_ptr(), None if v is None else v.data_ptr(),
                                       C.byref(step)))
        return step.value

    def nrc_forward(self, x, y):
        _check(_lib.pt_nrc_forward(self.h, x.data_ptr(), x.shape[0], y.data_ptr()))
        return y

    def nrc_gradient(self, x, t, grad):
        loss = C.c_double(0.0)
        _check(_lib.pt_nrc_gradient(self.h, x.data_ptr(), t.data_ptr(), x.shape[0], grad.data_ptr(), C.byref(loss)))
        return loss.value

    def nrc_train(self, x, t, frame, seed):
        loss = C.c_double(0.0)
        _check(_lib.pt_nrc_train(self.h, x.data_ptr(), t.data_ptr(), x.shape[0], frame, seed, C.byref(loss)))
        return loss.value

    def nrc_training_records(self, camera, frame, max_depth, seed, x, t, offsets=None):
        n = C.c_int64(0)
        _check(_lib.pt_nrc_training_records(self.h, C.byref(camera_struct(camera)), frame, max_depth, seed,
                                            x.data_ptr(), t.data_ptr(),
                                            None if offsets is None else offsets.data_ptr(), x.shape[0],
                                            C.byref(n)))
        return n.value

    def trace_closest(self, rays, hits, brute_force=False):
        _check(_lib.pt_trace_closest(self.h, rays.data_ptr(), rays.shape[0], hits.data_ptr(),
                                     1 if brute_force else 0))
        return hits

    def set_accumulation(self, sums, samples):
        """sums: float64 [h][w][3] device tensor holding the sums of `samples` samples per pixel."""
        _check(_lib.pt_set_accumulation(self.h, sums.data_ptr(), sums.shape[1], sums.shape[0], samples))

    def display(self, rgba8=None, encoded=None, exposure=1.0):
        """rgba8: uint8 [h][w][4] (or int32 [h][w]) device tensor; encoded: float32 [h][w][3]."""
        _check(_lib.pt_display(self.h, float(exposure), None if rgba8 is None else rgba8.data_ptr(),
                               None if encoded is None else encoded.data_ptr()))

    def trace_closest_noalloc(self, rays, hits, brute_force=False):
        _check(_lib.pt_trace_closest_noalloc(self.h, rays.data_ptr(), rays.shape[0], hits.data_ptr(),
                                             1 if brute_force else 0))
        return hits

    def stats(self) -> dict:
        st = pt_stats()
        _check(_lib.pt_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in pt_stats._fields_}

    def reset_stats(self):
        _check(_lib.pt_reset_stats(self.h))

    def set_tail(self, min_bounce=2, max_fraction=0.15):
        _check(_lib.pt_set_tail(self.h, int(min_bounce), float(max_fraction)))

    def set_profiling(self, timing: bool, counting: bool = False):
        _check(_lib.pt_set_profiling(self.h, 1 if timing else 0, 1 if counting else 0))


def scene_from(scene, device: int = 0, stream=None, gpu_bvh=False) -> PtScene:
    """Upload a scenes.Scene (geometry, materials, environment) to a new PtScene
    (BVH built on the host, or on the GPU with gpu_bvh: True or "ploc" for the
    default device builder, "lbvh" for the linear BVH)."""
    s = PtScene(device, stream)
    if isinstance(gpu_bvh, str):
        s.set_gpu_bvh_builder(gpu_bvh)
    s.build_bvh(scene.meshes, scene.instances, on_device=bool(gpu_bvh))
    s.upload_materials(scene.materials)
    s.set_environment(scene.env)
    return s


# ------------------------------------------------------------ host BVH --
class HostBvh:
    """pt_bvh_host_*: the BVH4 of one mesh built and walked on the CPU."""

    def __init__(self, mesh=None, meshes=None, instances=None):
        """HostBvh(mesh): one world-space mesh; HostBvh(meshes=..., instances=...): two levels."""
        keep = []
        h = C.c_void_p()
        if instances:
            arr = _mesh_structs(meshes, keep)
            ia = (pt_instance * len(instances))()
            for i, ins in enumerate(instances):
                ia[i].object_to_world[:] = [float(x) for x in np.asarray(ins.object_to_world, np.float32).reshape(12)]
                ia[i].mesh = int(ins.mesh)
                ia[i].material_override = int(ins.material_override)
            _check(_lib.pt_bvh_host_build_instanced(arr, len(meshes), ia, len(instances), C.byref(h)))
        else:
            arr = _mesh_structs([mesh], keep)
            _check(_lib.pt_bvh_host_build(arr, C.byref(h)))
        self.h = h
        info = pt_bvh_info()
        _check(_lib.pt_bvh_host_info(self.h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in pt_bvh_info._fields_}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pt_bvh_host_destroy(self.h)
        self.h = None

    def arrays(self):
        """(nodes uint8 [n,128], tris uint8 [n,48])"""
        nodes = np.zeros((self.info["n_nodes"], 128), dtype=np.uint8)
        tris = np.zeros((self.info["n_tris"], 48), dtype=np.uint8)
        _check(_lib.pt_bvh_host_copy(self.h, nodes.ctypes.data, tris.ctypes.data))
        return nodes, tris

    def trace(self, rays: np.ndarray) -> np.ndarray:
        rays = np.ascontiguousarray(rays, dtype=np.float32)
        hits = np.zeros((rays.shape[0], 6), dtype=np.uint32)
        _check(_lib.pt_bvh_host_trace(self.h, rays.ctypes.data, rays.shape[0], hits.ctypes.data))
        return hits

    def trace_stack(self, rays: np.ndarray, capacity: int = 0):
        """Host walk with a stack of `capacity` entries (0: the library's
        bound); returns (hits, deepest stack used).  Raises PTError on overflow."""
        rays = np.ascontiguousarray(rays, dtype=np.float32)
        hits = np.zeros((rays.shape[0], 6), dtype=np.uint32)
        high = C.c_int32(0)
        _check(_lib.pt_bvh_host_trace_stack(self.h, rays.ctypes.data, rays.shape[0], hits.ctypes.data, capacity,
                                            C.byref(high)))
        return hits, high.value
