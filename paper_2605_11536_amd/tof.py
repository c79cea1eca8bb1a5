"""Python binding of the ToF ReSTIR C ABI (include/tof.h).

Argument marshalling only: every step of the frame runs in the HIP library
``libtof.so`` built in this package.  PyTorch provides device memory and the
stream.  There is no fallback: a missing library or device raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtof.so")

TOF_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "invalid scene", -4: "not ready",
          -5: "device error", -6: "unimplemented"}

_i32p = C.POINTER(C.c_int32)
_f32p = C.POINTER(C.c_float)


class TofError(RuntimeError):
    def __init__(self, func: str, status: int):
        super().__init__(f"{func} failed: {STATUS.get(status, status)} ({status})")
        self.status = status


class tof_scene_desc(C.Structure):
    _fields_ = [("num_objects", C.c_int32), ("object_type", _i32p), ("object_material", _i32p),
                ("object_grid", _i32p), ("object_sphere", _f32p), ("num_materials", C.c_int32),
                ("material_type", _i32p), ("material_params", _f32p), ("num_vertices", C.c_int32),
                ("vertices", _f32p), ("scene_scale", C.c_float)]


class tof_sensor_desc(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("full_width", C.c_int32),
                ("full_height", C.c_int32), ("crop_x0", C.c_int32), ("crop_y0", C.c_int32),
                ("camera_model", C.c_int32), ("light_model", C.c_int32), ("count_camera_leg", C.c_int32),
                ("jitter", C.c_int32), ("light_intensity", C.c_float), ("gate_enabled", C.c_int32),
                ("gate_center", C.c_float), ("gate_width", C.c_float), ("n_bins", C.c_int32),
                ("bin_t0", C.c_float), ("bin_width", C.c_float), ("n_min", C.c_int32), ("n_max", C.c_int32),
                ("m_init", C.c_int32), ("temporal", C.c_int32), ("spatial_rounds", C.c_int32),
                ("spatial_k", C.c_int32), ("spatial_radius", C.c_int32), ("m_cap", C.c_float),
                ("newton_tol_rel", C.c_float), ("newton_max_iter", C.c_int32), ("j_max", C.c_float),
                ("shift_mode", C.c_int32), ("include_direct", C.c_int32), ("debug_stage", C.c_int32), ("bin_radius", C.c_int32),
                ("shrink_k", C.c_float), ("domain", C.c_int32), ("shrink_r", C.c_float),
                ("round_trip", C.c_int32), ("mis_mode", C.c_int32)]


class tof_launch_config(C.Structure):
    _fields_ = [("shift_blocks", C.c_uint32), ("vis_blocks", C.c_uint32), ("vis_waves", C.c_uint32),
                ("merge_tasks", C.c_uint32)]


def _launch_dict(cfg) -> dict:
    return {"shift_blocks": int(cfg.shift_blocks), "vis_blocks": int(cfg.vis_blocks),
            "vis_waves": int(cfg.vis_waves), "merge_tasks": int(cfg.merge_tasks)}


class tof_bvh_info(C.Structure):
    _fields_ = [("builder", C.c_int32), ("num_nodes", C.c_int32), ("num_levels", C.c_int32), ("rounds", C.c_int32),
                ("num_triangles", C.c_int32), ("pad", C.c_int32), ("build_ms", C.c_double)]


BVH_HOST, BVH_DEVICE = 0, 1


class tof_frame_desc(C.Structure):
    _fields_ = [("frame_index", C.c_int32), ("cam_pos", C.c_float * 3), ("cam_fwd", C.c_float * 3),
                ("cam_up", C.c_float * 3), ("fov_y_deg", C.c_float), ("ortho_half", C.c_float * 2),
                ("light_pos", C.c_float * 3), ("object_xforms", _f32p), ("object_velocities", _f32p),
                ("cam_vel", C.c_float * 3), ("light_vel", C.c_float * 3)]


class tof_history_desc(C.Structure):
    _fields_ = [("W", _f32p), ("phat", _f32p), ("len", _f32p), ("pre_pdf", _f32p),
                ("origin_pixel", C.POINTER(C.c_uint32)), ("origin_frame", C.POINTER(C.c_uint32)),
                ("meta", C.POINTER(C.c_uint32)), ("vertex_obj", _i32p), ("vertex_xi", _f32p), ("M", _f32p),
                ("mask", C.POINTER(C.c_uint32))]


KERNELS = ("bvh", "gbuffer", "initial", "temporal_prep", "temporal_fwd", "temporal_mis", "temporal_vis",
           "temporal_merge", "spatial_prep", "spatial_fwd", "spatial_mis", "spatial_vis", "spatial_merge", "splat")


WORK_FIELDS = ("rays", "node_visits", "tri_tests", "shifts", "newton_attempts", "newton_iters")


class tof_kernel_work(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in WORK_FIELDS]


class tof_kernel_times(C.Structure):
    _fields_ = [("ms", C.c_double * len(KERNELS)), ("launches", C.c_uint64 * len(KERNELS)),
                ("work_items", C.c_uint64 * 4), ("work", tof_kernel_work * len(KERNELS))]


class tof_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("shifts", "shifts_ok", "newton_attempts", "newton_converged",
                                          "newton_iters", "newton_paths_ok", "rays", "frames", "bvh_overflow",
                                          "node_visits", "tri_tests", "bad_records")]


_lib = None


def lib():
    """Load libtof.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.tof_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_size_t, C.c_uint64]
        L.tof_destroy.argtypes = [C.c_void_p]
        L.tof_destroy.restype = None
        L.tof_scene_upload.argtypes = [C.c_void_p, C.POINTER(tof_scene_desc)]
        L.tof_sensor_set.argtypes = [C.c_void_p, C.POINTER(tof_sensor_desc)]
        L.tof_render_frame.argtypes = [C.c_void_p, C.POINTER(tof_frame_desc), C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
        L.tof_render_frame_noalloc.argtypes = [C.c_void_p, C.POINTER(tof_frame_desc), C.c_void_p, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.c_void_p]
        L.tof_render_frame_noalloc.restype = C.c_int
        L.tof_reservoirs_reset.argtypes = [C.c_void_p]
        L.tof_get_stats.argtypes = [C.c_void_p, C.POINTER(tof_stats)]
        L.tof_debug_set_ray_budget.argtypes = [C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.tof_debug_set_ray_budget.restype = C.c_int
        L.tof_debug_set_history.argtypes = [C.c_void_p, C.POINTER(tof_history_desc)]
        L.tof_debug_set_history.restype = C.c_int
        L.tof_set_launch_config.argtypes = [C.c_void_p, C.POINTER(tof_launch_config)]
        L.tof_get_launch_config.argtypes = [C.c_void_p, C.POINTER(tof_launch_config)]
        L.tof_autotune.argtypes = [C.c_void_p, C.POINTER(tof_frame_desc), C.c_int, C.c_void_p,
                                   C.POINTER(tof_launch_config)]
        L.tof_set_bvh_builder.argtypes = [C.c_void_p, C.c_int32]
        L.tof_get_bvh_info.argtypes = [C.c_void_p, C.POINTER(tof_bvh_info), C.c_void_p]
        for f in ("tof_set_launch_config", "tof_get_launch_config", "tof_autotune", "tof_set_bvh_builder",
                  "tof_get_bvh_info"):
            getattr(L, f).restype = C.c_int
        L.tof_set_kernel_timing.argtypes = [C.c_void_p, C.c_int]
        L.tof_set_kernel_timing.restype = C.c_int
        L.tof_get_kernel_times.argtypes = [C.c_void_p, C.POINTER(tof_kernel_times)]
        L.tof_get_kernel_times.restype = C.c_int
        L.tof_status_string.argtypes = [C.c_int]
        L.tof_status_string.restype = C.c_char_p
        L.tof_footprint.argtypes = [C.POINTER(tof_scene_desc), C.POINTER(tof_sensor_desc), C.POINTER(C.c_size_t)]
        L.tof_server_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_size_t]
        L.tof_server_destroy.argtypes = [C.c_void_p]
        L.tof_server_destroy.restype = None
        L.tof_server_open.argtypes = [C.c_void_p, C.POINTER(tof_scene_desc), C.POINTER(tof_sensor_desc), C.c_uint64,
                                      C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.tof_server_submit.argtypes = [C.c_void_p, C.c_int, C.POINTER(tof_frame_desc), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]
        L.tof_server_query.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]
        L.tof_server_query_timed.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_float)]
        L.tof_server_query_timed.restype = C.c_int
        L.tof_server_wait.argtypes = [C.c_void_p, C.c_uint64]
        L.tof_server_close.argtypes = [C.c_void_p, C.c_int]
        L.tof_server_info.argtypes = [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.tof_server_set_graphs.argtypes = [C.c_void_p, C.c_int]
        L.tof_server_set_graphs.restype = C.c_int
        for f in ("tof_footprint", "tof_server_create", "tof_server_open", "tof_server_submit", "tof_server_query",
                  "tof_server_wait", "tof_server_close", "tof_server_info"):
            getattr(L, f).restype = C.c_int
        for f in ("tof_create", "tof_scene_upload", "tof_sensor_set", "tof_render_frame",
                  "tof_reservoirs_reset", "tof_get_stats"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(func: str, st: int):
    if st != TOF_OK:
        raise TofError(func, st)


def _ptr(a, t):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------------------
# the C entry points, one Python function each
# ---------------------------------------------------------------------------

def tof_create(device: int = 0, hbm_budget_bytes: int = 0, seed: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    _check("tof_create", lib().tof_create(C.byref(h), int(device), int(hbm_budget_bytes), int(seed)))
    return h


def tof_destroy(h) -> None:
    if h:
        lib().tof_destroy(h)


def scene_desc(scene):
    """The C description of a scene and the arrays it points into (keep both)."""
    arrs = dict(
        t=np.ascontiguousarray(scene.obj_type, dtype=np.int32),
        m=np.ascontiguousarray(scene.obj_material, dtype=np.int32),
        g=np.ascontiguousarray(scene.obj_grid, dtype=np.int32),
        s=np.ascontiguousarray(scene.obj_sphere, dtype=np.float32),
        mt=np.ascontiguousarray(scene.mat_type, dtype=np.int32),
        mp=np.ascontiguousarray(scene.mat_params, dtype=np.float32),
        v=np.ascontiguousarray(scene.vertices, dtype=np.float32),
    )
    d = tof_scene_desc(int(arrs["t"].shape[0]), _ptr(arrs["t"], _i32p), _ptr(arrs["m"], _i32p),
                       _ptr(arrs["g"], _i32p), _ptr(arrs["s"], _f32p), int(arrs["mt"].shape[0]),
                       _ptr(arrs["mt"], _i32p), _ptr(arrs["mp"], _f32p), int(arrs["v"].shape[0]),
                       _ptr(arrs["v"], _f32p), float(scene.scene_scale))
    return d, arrs


def tof_scene_upload(h, scene) -> None:
    d, _arrs = scene_desc(scene)
    _check("tof_scene_upload", lib().tof_scene_upload(h, C.byref(d)))


def tof_footprint(scene, sensor) -> int:
    d, _arrs = scene_desc(scene)
    sd = sensor_desc(sensor)
    n = C.c_size_t(0)
    _check("tof_footprint", lib().tof_footprint(C.byref(d), C.byref(sd), C.byref(n)))
    return int(n.value)


def sensor_desc(sensor) -> tof_sensor_desc:
    d = tof_sensor_desc()
    for name, _ in tof_sensor_desc._fields_:
        setattr(d, name, getattr(sensor, name))
    return d


def tof_sensor_set(h, sensor) -> None:
    d = sensor_desc(sensor)
    _check("tof_sensor_set", lib().tof_sensor_set(h, C.byref(d)))


def frame_desc(frame):
    d = tof_frame_desc()
    d.frame_index = int(frame.index)
    for i in range(3):
        d.cam_pos[i] = float(frame.cam_pos[i])
        d.cam_fwd[i] = float(frame.cam_fwd[i])
        d.cam_up[i] = float(frame.cam_up[i])
        d.light_pos[i] = float(frame.light_pos[i])
    d.fov_y_deg = float(frame.fov_y_deg)
    d.ortho_half[0] = float(frame.ortho_half[0])
    d.ortho_half[1] = float(frame.ortho_half[1])
    xf = np.ascontiguousarray(frame.xforms, dtype=np.float32)
    d.object_xforms = _ptr(xf, _f32p)
    vel = None
    if getattr(frame, "velocities", None) is not None:
        vel = np.ascontiguousarray(frame.velocities, dtype=np.float32)
        d.object_velocities = _ptr(vel, _f32p)
    for i in range(3):
        d.cam_vel[i] = float(getattr(frame, "cam_vel", (0.0, 0.0, 0.0))[i])
        d.light_vel[i] = float(getattr(frame, "light_vel", (0.0, 0.0, 0.0))[i])
    return d, (xf, vel)


def _dptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def tof_render_frame(h, frame, out_image=None, out_hist=None, out_pt_image=None, out_pt_hist=None,
                     stream=None) -> None:
    """Outputs are float32 CUDA/HIP torch tensors (or None); stream is a
    torch.cuda.Stream (None = torch's current stream)."""
    import torch
    for t in (out_image, out_hist, out_pt_image, out_pt_hist):
        if t is not None:
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    if stream is None:
        stream = torch.cuda.current_stream()
    d, xf = frame_desc(frame)
    _check("tof_render_frame", lib().tof_render_frame(h, C.byref(d), _dptr(out_image), _dptr(out_hist),
                                                      _dptr(out_pt_image), _dptr(out_pt_hist),
                                                      C.c_void_p(stream.cuda_stream)))


def tof_render_frame_noalloc(h, frame, out_image=None, out_hist=None, out_pt_image=None, out_pt_hist=None,
                             stream=None) -> None:
    """tof_render_frame with the frame's work space in the library's static
    device array (allocates nothing)."""
    import torch
    for t in (out_image, out_hist, out_pt_image, out_pt_hist):
        if t is not None:
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    if stream is None:
        stream = torch.cuda.current_stream()
    d, xf = frame_desc(frame)
    _check("tof_render_frame_noalloc",
           lib().tof_render_frame_noalloc(h, C.byref(d), _dptr(out_image), _dptr(out_hist), _dptr(out_pt_image),
                                          _dptr(out_pt_hist), C.c_void_p(stream.cuda_stream)))


def tof_set_launch_config(h, shift_blocks: int = 0, vis_blocks: int = 0, vis_waves: int = 0,
                          merge_tasks: int = 0) -> None:
    cfg = tof_launch_config(int(shift_blocks), int(vis_blocks), int(vis_waves), int(merge_tasks))
    _check("tof_set_launch_config", lib().tof_set_launch_config(h, C.byref(cfg)))


def tof_get_launch_config(h) -> dict:
    cfg = tof_launch_config()
    _check("tof_get_launch_config", lib().tof_get_launch_config(h, C.byref(cfg)))
    return _launch_dict(cfg)


def tof_set_bvh_builder(h, builder: int) -> None:
    _check("tof_set_bvh_builder", lib().tof_set_bvh_builder(h, int(builder)))


def tof_get_bvh_info(h, leaf_triangles: bool = False):
    """The last scene upload's tree summary as a dict, and with
    leaf_triangles the triangle of every leaf slot (numpy int32)."""
    info = tof_bvh_info()
    _check("tof_get_bvh_info", lib().tof_get_bvh_info(h, C.byref(info), None))
    out = {"builder": int(info.builder), "num_nodes": int(info.num_nodes), "num_levels": int(info.num_levels),
           "rounds": int(info.rounds), "num_triangles": int(info.num_triangles), "build_ms": float(info.build_ms)}
    if leaf_triangles:
        arr = np.zeros(max(info.num_triangles, 0), np.int32)
        _check("tof_get_bvh_info", lib().tof_get_bvh_info(h, C.byref(info), arr.ctypes.data_as(C.c_void_p)))
        out["leaf_triangles"] = arr
    return out


def tof_autotune(h, frames, stream=None) -> dict:
    """Time the candidate launch shapes over `frames` (a list of Frame) and
    keep the fastest; returns it."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    descs, keep = [], []
    for fr in frames:
        d, k = frame_desc(fr)
        descs.append(d)
        keep.append(k)
    arr = (tof_frame_desc * len(descs))(*descs)
    cfg = tof_launch_config()
    _check("tof_autotune", lib().tof_autotune(h, arr, len(descs), C.c_void_p(stream.cuda_stream), C.byref(cfg)))
    return _launch_dict(cfg)


def tof_reservoirs_reset(h) -> None:
    _check("tof_reservoirs_reset", lib().tof_reservoirs_reset(h))


def tof_get_stats(h) -> dict:
    s = tof_stats()
    _check("tof_get_stats", lib().tof_get_stats(h, C.byref(s)))
    return {name: int(getattr(s, name)) for name, _ in tof_stats._fields_}


def tof_debug_set_history(h, hist: dict) -> None:
    """hist: numpy arrays W, phat, len, pre_pdf (f32), opix, ofr, meta (u32),
    vobj (i32, 4*P*B), vxi (f32, 8*P*B), M (f32, P), mask (u32)."""
    u32 = C.POINTER(C.c_uint32)
    types = dict(W=np.float32, phat=np.float32, len=np.float32, pre_pdf=np.float32, opix=np.uint32,
                 ofr=np.uint32, meta=np.uint32, vobj=np.int32, vxi=np.float32, M=np.float32, mask=np.uint32)
    # converted arrays stay referenced by `a` until the call returns
    a = {k: np.ascontiguousarray(hist[k], dtype=t) for k, t in types.items()}
    d = tof_history_desc(_ptr(a["W"], _f32p), _ptr(a["phat"], _f32p), _ptr(a["len"], _f32p),
                         _ptr(a["pre_pdf"], _f32p), _ptr(a["opix"], u32), _ptr(a["ofr"], u32),
                         _ptr(a["meta"], u32), _ptr(a["vobj"], _i32p), _ptr(a["vxi"], _f32p),
                         _ptr(a["M"], _f32p), _ptr(a["mask"], u32))
    _check("tof_debug_set_history", lib().tof_debug_set_history(h, C.byref(d)))


def tof_set_kernel_timing(h, enabled: bool) -> None:
    _check("tof_set_kernel_timing", lib().tof_set_kernel_timing(h, int(bool(enabled))))


def tof_get_kernel_times(h) -> dict:
    t = tof_kernel_times()
    _check("tof_get_kernel_times", lib().tof_get_kernel_times(h, C.byref(t)))
    out = {k: {"ms": float(t.ms[i]), "launches": int(t.launches[i]),
               "work": {n: int(getattr(t.work[i], n)) for n in WORK_FIELDS}} for i, k in enumerate(KERNELS)}
    out["work_items"] = {"temporal_items": int(t.work_items[0]), "temporal_tasks": int(t.work_items[1]),
                         "spatial_items": int(t.work_items[2]), "spatial_tasks": int(t.work_items[3])}
    return out


def tof_status_string(status: int) -> str:
    return lib().tof_status_string(int(status)).decode()


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

class Renderer:
    """One render stream: a context with a scene and a sensor."""

    def __init__(self, scene, sensor, device: int = 0, hbm_budget_bytes: int = 0, bvh_builder: int = BVH_HOST):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the ToF ReSTIR library runs on HIP devices only")
        self.device = torch.device("cuda", device)
        self.sensor = sensor
        self.h = tof_create(device, hbm_budget_bytes, sensor.seed)
        tof_set_bvh_builder(self.h, bvh_builder)
        tof_scene_upload(self.h, scene)
        tof_sensor_set(self.h, sensor)
        P = sensor.width * sensor.height
        self.out_image = torch.zeros(P, dtype=torch.float32, device=self.device) if sensor.gate_enabled else None
        self.out_pt_image = torch.zeros(P, dtype=torch.float32, device=self.device) if sensor.gate_enabled else None
        nb = sensor.n_bins
        self.out_hist = torch.zeros(nb * P, dtype=torch.float32, device=self.device) if nb else None
        self.out_pt_hist = torch.zeros(nb * P, dtype=torch.float32, device=self.device) if nb else None

    def render(self, frame, stream=None):
        tof_render_frame(self.h, frame, self.out_image, self.out_hist, self.out_pt_image, self.out_pt_hist,
                         stream)

    def render_noalloc(self, frame, stream=None):
        tof_render_frame_noalloc(self.h, frame, self.out_image, self.out_hist, self.out_pt_image, self.out_pt_hist,
                                 stream)

    def fetch(self) -> dict:
        import torch
        torch.cuda.synchronize(self.device)
        s = self.sensor
        shp = (s.height, s.width)
        out = {}
        if self.out_image is not None:
            out["image"] = self.out_image.cpu().numpy().reshape(shp)
            out["pt_image"] = self.out_pt_image.cpu().numpy().reshape(shp)
        if self.out_hist is not None:
            out["hist"] = self.out_hist.cpu().numpy().reshape((s.n_bins,) + shp)
            out["pt_hist"] = self.out_pt_hist.cpu().numpy().reshape((s.n_bins,) + shp)
        return out

    def stats(self) -> dict:
        return tof_get_stats(self.h)

    def reset(self):
        tof_reservoirs_reset(self.h)

    def set_gate_center(self, center: float):
        """Move the gate, keeping the history (tof_sensor_set with only the
        centre changed)."""
        import dataclasses
        self.sensor = dataclasses.replace(self.sensor, gate_center=float(center))
        tof_sensor_set(self.h, self.sensor)

    def set_kernel_timing(self, enabled: bool):
        tof_set_kernel_timing(self.h, enabled)

    def kernel_times(self) -> dict:
        return tof_get_kernel_times(self.h)

    def set_ray_budget(self, rays: int) -> int:
        """Test support: chunks of the reuse passes sized to `rays` visibility
        rays (0 = default); returns the items per spatial chunk."""
        n = C.c_size_t(0)
        _check("tof_debug_set_ray_budget", lib().tof_debug_set_ray_budget(self.h, int(rays), C.byref(n)))
        return int(n.value)

    def set_history(self, hist: dict):
        tof_debug_set_history(self.h, hist)

    def set_launch_config(self, shift_blocks: int = 0, vis_blocks: int = 0, vis_waves: int = 0,
                          merge_tasks: int = 0):
        tof_set_launch_config(self.h, shift_blocks, vis_blocks, vis_waves, merge_tasks)

    def launch_config(self) -> dict:
        return tof_get_launch_config(self.h)

    def autotune(self, frames, stream=None) -> dict:
        return tof_autotune(self.h, frames, stream)

    def upload_scene(self, scene, bvh_builder: int = None):
        """Replace the scene (drops the temporal history); bvh_builder
        BVH_HOST or BVH_DEVICE, else the context's current choice."""
        if bvh_builder is not None:
            tof_set_bvh_builder(self.h, bvh_builder)
        tof_scene_upload(self.h, scene)

    def bvh_info(self, leaf_triangles: bool = False) -> dict:
        return tof_get_bvh_info(self.h, leaf_triangles)

    def close(self):
        if self.h:
            tof_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# serving (tof_server_*): argument marshalling only
# ---------------------------------------------------------------------------
class Server:
    """Request loop over render streams on one device (see include/tof.h)."""

    def __init__(self, hbm_budget_bytes: int, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the ToF ReSTIR library runs on HIP devices only")
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        _check("tof_server_create", lib().tof_server_create(C.byref(h), device, int(hbm_budget_bytes)))
        self.h = h
        self.sensors = {}

    def open(self, scene, sensor):
        """Returns (stream id, admitted now)."""
        d, _arrs = scene_desc(scene)
        sd = sensor_desc(sensor)
        sid, adm = C.c_int(-1), C.c_int(0)
        _check("tof_server_open", lib().tof_server_open(self.h, C.byref(d), C.byref(sd), int(sensor.seed),
                                                         C.byref(sid), C.byref(adm)))
        self.sensors[sid.value] = sensor
        return sid.value, bool(adm.value)

    def outputs(self, sid, pt: bool = True):
        """Output tensors for frames of stream sid (pt: also the plain-PT
        outputs).  They are left uninitialised: the splat writes every
        element, and no fill kernel on torch's stream may race with the
        server's stream that writes them."""
        import torch
        s = self.sensors[sid]
        P = s.width * s.height
        e = lambda n: torch.empty(n, dtype=torch.float32, device=self.device)   # noqa: E731
        out = {"image": e(P) if s.gate_enabled else None, "hist": e(s.n_bins * P) if s.n_bins else None,
               "pt_image": e(P) if s.gate_enabled and pt else None,
               "pt_hist": e(s.n_bins * P) if s.n_bins and pt else None}
        # the blocks may come back from tensors whose last use is still queued
        # on torch's stream, which the server's streams do not wait for
        torch.cuda.current_stream(self.device).synchronize()
        return out

    def submit(self, sid, frame, out) -> int:
        d, _xf = frame_desc(frame)
        t = C.c_uint64(0)
        _check("tof_server_submit", lib().tof_server_submit(self.h, sid, C.byref(d), _dptr(out["image"]),
                                                             _dptr(out["hist"]), _dptr(out["pt_image"]),
                                                             _dptr(out["pt_hist"]), C.byref(t)))
        return int(t.value)

    def query(self, ticket) -> bool:
        done = C.c_int(0)
        _check("tof_server_query", lib().tof_server_query(self.h, C.c_uint64(ticket), C.byref(done)))
        return bool(done.value)

    def query_timed(self, ticket):
        """(done, GPU service time in ms of the frame once done, else None)."""
        done, ms = C.c_int(0), C.c_float(-1.0)
        _check("tof_server_query_timed",
               lib().tof_server_query_timed(self.h, C.c_uint64(ticket), C.byref(done), C.byref(ms)))
        return bool(done.value), (float(ms.value) if done.value and ms.value >= 0 else None)

    def wait(self, ticket) -> None:
        _check("tof_server_wait", lib().tof_server_wait(self.h, C.c_uint64(ticket)))

    def close_stream(self, sid) -> None:
        _check("tof_server_close", lib().tof_server_close(self.h, sid))
        self.sensors.pop(sid, None)

    def set_graphs(self, enabled: bool) -> None:
        """Record each later frame into a HIP graph and launch it as one."""
        _check("tof_server_set_graphs", lib().tof_server_set_graphs(self.h, 1 if enabled else 0))

    def info(self) -> dict:
        used, adm, wait = C.c_size_t(0), C.c_int(0), C.c_int(0)
        _check("tof_server_info", lib().tof_server_info(self.h, C.byref(used), C.byref(adm), C.byref(wait)))
        return {"used_bytes": int(used.value), "admitted": adm.value, "waiting": wait.value}

    @staticmethod
    def fetch(sensor, out) -> dict:
        shp = (sensor.height, sensor.width)
        res = {}
        for k in ("image", "pt_image"):
            if out[k] is not None:
                res[k] = out[k].cpu().numpy().reshape(shp)
        for k in ("hist", "pt_hist"):
            if out[k] is not None:
                res[k] = out[k].cpu().numpy().reshape((sensor.n_bins,) + shp)
        return res

    def close(self):
        if self.h is not None:
            lib().tof_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
