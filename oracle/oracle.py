"""ctypes wrapper of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and bench.py's CPU-baseline leg may import this.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_i32p = C.POINTER(C.c_int32)
_f32p = C.POINTER(C.c_float)
_f64p = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)


class OrcScene(C.Structure):
    _fields_ = [("num_objects", C.c_int32), ("obj_type", _i32p), ("obj_material", _i32p),
                ("obj_grid", _i32p), ("obj_sphere", _f32p), ("num_materials", C.c_int32),
                ("mat_type", _i32p), ("mat_params", _f32p), ("num_vertices", C.c_int32),
                ("vertices", _f32p), ("scene_scale", C.c_float)]


class OrcSensor(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("full_width", C.c_int32),
                ("full_height", C.c_int32), ("crop_x0", C.c_int32), ("crop_y0", C.c_int32),
                ("camera_model", C.c_int32), ("light_model", C.c_int32),
                ("count_camera_leg", C.c_int32), ("jitter", C.c_int32),
                ("light_intensity", C.c_double), ("gate_enabled", C.c_int32),
                ("gate_center", C.c_double), ("gate_width", C.c_double), ("n_bins", C.c_int32),
                ("bin_t0", C.c_double), ("bin_width", C.c_double), ("n_min", C.c_int32),
                ("n_max", C.c_int32), ("m_init", C.c_int32), ("temporal", C.c_int32),
                ("spatial_rounds", C.c_int32), ("spatial_k", C.c_int32),
                ("spatial_radius", C.c_int32), ("m_cap", C.c_double),
                ("newton_tol_rel", C.c_double), ("newton_max_iter", C.c_int32),
                ("j_max", C.c_double), ("shift_mode", C.c_int32), ("include_direct", C.c_int32),
                ("debug_stage", C.c_int32), ("bin_radius", C.c_int32),
                ("shrink_k", C.c_double), ("shrink_r", C.c_double), ("domain", C.c_int32), ("round_trip", C.c_int32), ("mis_mode", C.c_int32),
                ("seed", C.c_uint64)]


class OrcFrame(C.Structure):
    _fields_ = [("index", C.c_int32), ("cam_pos", C.c_float * 3), ("cam_fwd", C.c_float * 3),
                ("cam_up", C.c_float * 3), ("fov_y_deg", C.c_float), ("ortho_half", C.c_float * 2),
                ("light_pos", C.c_float * 3), ("xforms", _f32p), ("velocities", _f32p),
                ("cam_vel", C.c_float * 3), ("light_vel", C.c_float * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _build
            _build.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_create.restype = C.c_void_p
        _lib.orc_create.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcSensor), C.c_int]
        _lib.orc_destroy.argtypes = [C.c_void_p]
        _lib.orc_reset.argtypes = [C.c_void_p]
        _lib.orc_set_gate_center.argtypes = [C.c_void_p, C.c_double]
        _lib.orc_render_frame.argtypes = [C.c_void_p, C.POINTER(OrcFrame), _f64p, _f64p, _f64p, _f64p]
        _lib.orc_get_stats.argtypes = [C.c_void_p, _u64p]
        _lib.orc_get_merge_diag.argtypes = [C.c_void_p, _f64p]
        _lib.orc_philox4x64.argtypes = [_u64p, _u64p, _u64p]
        _lib.orc_load_frame.argtypes = [C.c_void_p, C.POINTER(OrcFrame)]
        _lib.orc_trace.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, _f64p]
        _lib.orc_chart.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p]
        _lib.orc_newton.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p, _f64p, C.c_double, _f64p, _f64p,
                                    C.c_double, C.c_double, C.c_double, C.c_int, _f64p]
        _u32p = C.POINTER(C.c_uint32)
        _lib.orc_export_history.argtypes = [C.c_void_p, _f32p, _f32p, _f32p, _f32p, _u32p, _u32p, _u32p, _i32p,
                                            _f32p, _f32p, _u32p]
        _lib.orc_vel_eval.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p, _f64p, _f64p, _f64p, C.c_double,
                                      _f64p]
        _lib.orc_occluded.restype = C.c_int
        _lib.orc_occluded.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double]
        _lib.orc_bsdf.restype = None
        _lib.orc_bsdf.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p, _f64p, C.c_int, _f64p]
        _lib.orc_bsdf_sample.restype = C.c_int
        _lib.orc_bsdf_sample.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p, _f64p, C.c_int, _f64p, _f64p]
        _lib.orc_mis_weights.restype = None
        _lib.orc_mis_weights.argtypes = [C.c_int, C.c_int, _f64p, C.c_double, _f64p, C.c_double, _f64p]
        _lib.orc_wrs.restype = C.c_int
        _lib.orc_wrs.argtypes = [_f64p, _f64p, C.c_int, _f64p]
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_f64p)


def philox4x64(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_p(c, _u64p), _p(k, _u64p), _p(o, _u64p))
    return o


def wrs(w, u):
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    ws = C.c_double(0.0)
    sel = lib().orc_wrs(_p(w, _f64p), _p(u, _f64p), len(w), C.byref(ws))
    return sel, ws.value


def mis_weights(mode, M, mq, d, dc):
    """MIS weights [canonical, neighbour 0..K-1] of the spatial reuse at one path."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(len(M) + 1)
    lib().orc_mis_weights(int(mode), len(M), _p(M, _f64p), float(mq), _p(d, _f64p), float(dc), _p(out, _f64p))
    return out


def make_frame(fr):
    f = OrcFrame()
    f.index = int(fr.index)
    for i in range(3):
        f.cam_pos[i] = float(fr.cam_pos[i])
        f.cam_fwd[i] = float(fr.cam_fwd[i])
        f.cam_up[i] = float(fr.cam_up[i])
        f.light_pos[i] = float(fr.light_pos[i])
    f.fov_y_deg = float(fr.fov_y_deg)
    f.ortho_half[0] = float(fr.ortho_half[0])
    f.ortho_half[1] = float(fr.ortho_half[1])
    xf = np.ascontiguousarray(fr.xforms, dtype=np.float32)
    f.xforms = _p(xf, _f32p)
    vel = None
    if getattr(fr, "velocities", None) is not None:
        vel = np.ascontiguousarray(fr.velocities, dtype=np.float32)
        f.velocities = _p(vel, _f32p)
    for i in range(3):
        f.cam_vel[i] = float(getattr(fr, "cam_vel", (0.0, 0.0, 0.0))[i])
        f.light_vel[i] = float(getattr(fr, "light_vel", (0.0, 0.0, 0.0))[i])
    return f, (xf, vel)


class Oracle:
    """One oracle render stream over a scenes.Workload-shaped scene/sensor."""

    def __init__(self, scene, sensor, num_threads=None):
        self._keep = []
        sc = OrcScene()
        arrs = dict(
            obj_type=np.ascontiguousarray(scene.obj_type, dtype=np.int32),
            obj_material=np.ascontiguousarray(scene.obj_material, dtype=np.int32),
            obj_grid=np.ascontiguousarray(scene.obj_grid, dtype=np.int32),
            obj_sphere=np.ascontiguousarray(scene.obj_sphere, dtype=np.float32),
            mat_type=np.ascontiguousarray(scene.mat_type, dtype=np.int32),
            mat_params=np.ascontiguousarray(scene.mat_params, dtype=np.float32),
            vertices=np.ascontiguousarray(scene.vertices, dtype=np.float32),
        )
        self._keep.append(arrs)
        sc.num_objects = scene.num_objects
        sc.obj_type = _p(arrs["obj_type"], _i32p)
        sc.obj_material = _p(arrs["obj_material"], _i32p)
        sc.obj_grid = _p(arrs["obj_grid"], _i32p)
        sc.obj_sphere = _p(arrs["obj_sphere"], _f32p)
        sc.num_materials = int(arrs["mat_type"].shape[0])
        sc.mat_type = _p(arrs["mat_type"], _i32p)
        sc.mat_params = _p(arrs["mat_params"], _f32p)
        sc.num_vertices = int(arrs["vertices"].shape[0])
        sc.vertices = _p(arrs["vertices"], _f32p)
        sc.scene_scale = scene.scene_scale
        sn = OrcSensor()
        for name, t in OrcSensor._fields_:
            v = getattr(sensor, name)
            if t is C.c_double:   # the same float32 value the HIP library receives
                v = float(np.float32(v))
            setattr(sn, name, v)
        self.sensor = sensor
        nt = num_threads or os.cpu_count() or 1
        self.num_threads = nt
        self.h = lib().orc_create(C.byref(sc), C.byref(sn), int(nt))
        if not self.h:
            raise ValueError("sensor rejected by the oracle (an unsupported combination of settings)")

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        lib().orc_reset(self.h)

    def set_gate_center(self, center: float):
        """Move the gate, keeping the history (Sec. 4.1 time-gate shifting)."""
        import dataclasses
        c = float(np.float32(center))
        self.sensor = dataclasses.replace(self.sensor, gate_center=c)
        lib().orc_set_gate_center(self.h, c)

    def render(self, frame):
        s = self.sensor
        P = s.width * s.height
        img = np.zeros(P) if s.gate_enabled else None
        pimg = np.zeros(P) if s.gate_enabled else None
        hist = np.zeros(s.n_bins * P) if s.n_bins else None
        phist = np.zeros(s.n_bins * P) if s.n_bins else None
        f, xf = make_frame(frame)
        rc = lib().orc_render_frame(self.h, C.byref(f), _dp(img), _dp(hist), _dp(pimg), _dp(phist))
        assert rc == 0
        shp = (s.height, s.width)
        out = {}
        if img is not None:
            out["image"] = img.reshape(shp)
            out["pt_image"] = pimg.reshape(shp)
        if hist is not None:
            out["hist"] = hist.reshape((s.n_bins,) + shp)
            out["pt_hist"] = phist.reshape((s.n_bins,) + shp)
        return out

    def stats(self):
        o = np.zeros(8, dtype=np.uint64)
        lib().orc_get_stats(self.h, _p(o, _u64p))
        keys = ["shifts", "shifts_ok", "newton_attempts", "newton_converged", "newton_iters",
                "newton_paths_ok", "rays", "reserved"]
        return {k: int(v) for k, v in zip(keys, o)}

    def merge_diag(self):
        """Sums over the merges so far, per pass ("temporal", "spatial"):
        merges, ess (effective sample count), positive (candidates with w > 0),
        present (non-empty candidate reservoirs) and canonical_share."""
        o = np.zeros(10, dtype=np.float64)
        lib().orc_get_merge_diag(self.h, _p(o, _f64p))
        keys = ["merges", "ess", "positive", "present", "canonical_share"]
        return {name: {k: float(v) for k, v in zip(keys, o[5 * i:5 * i + 5])}
                for i, name in enumerate(("temporal", "spatial"))}

    def export_history(self):
        """Final reservoirs of the last frame (float32 SoA, plane-major)."""
        s = self.sensor
        P, B = s.width * s.height, s.n_bins + (1 if s.gate_enabled else 0)
        PB = P * B
        h = dict(W=np.zeros(PB, np.float32), phat=np.zeros(PB, np.float32), len=np.zeros(PB, np.float32),
                 pre_pdf=np.zeros(PB, np.float32), opix=np.zeros(PB, np.uint32), ofr=np.zeros(PB, np.uint32),
                 meta=np.zeros(PB, np.uint32), vobj=np.full(4 * PB, -1, np.int32), vxi=np.zeros(8 * PB, np.float32),
                 M=np.zeros(P, np.float32), mask=np.zeros(((B + 31) // 32) * P, np.uint32))
        u32 = C.POINTER(C.c_uint32)
        rc = lib().orc_export_history(self.h, _p(h["W"], _f32p), _p(h["phat"], _f32p), _p(h["len"], _f32p),
                                      _p(h["pre_pdf"], _f32p), _p(h["opix"], u32), _p(h["ofr"], u32),
                                      _p(h["meta"], u32), _p(h["vobj"], _i32p), _p(h["vxi"], _f32p),
                                      _p(h["M"], _f32p), _p(h["mask"], u32))
        assert rc == 0, "no history"
        return h

    # unit-level helpers
    def load_frame(self, frame):
        f, xf = make_frame(frame)
        lib().orc_load_frame(self.h, C.byref(f))

    def trace(self, o, d, brute=False):
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        out = np.zeros(4)
        prim = lib().orc_trace(self.h, _p(o, _f64p), _p(d, _f64p), int(brute), _p(out, _f64p))
        return prim, out

    def occluded(self, o, d, tmax):
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        return bool(lib().orc_occluded(self.h, _p(o, _f64p), _p(d, _f64p), float(tmax)))

    def bsdf(self, obj, n, wi, wo):
        """f_s(wi, wo) for directions wo [N, 3]."""
        n = np.ascontiguousarray(n, dtype=np.float64)
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        wo = np.ascontiguousarray(np.reshape(wo, (-1, 3)), dtype=np.float64)
        out = np.zeros(wo.shape[0])
        lib().orc_bsdf(self.h, int(obj), _p(n, _f64p), _p(wi, _f64p), _p(wo, _f64p), wo.shape[0], _p(out, _f64p))
        return out

    def bsdf_sample(self, obj, n, wi, u):
        """Sampled directions [N, 3] and densities [N] (0 = rejected) for uniforms u [N, 2]."""
        n = np.ascontiguousarray(n, dtype=np.float64)
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        u = np.ascontiguousarray(np.reshape(u, (-1, 2)), dtype=np.float64)
        wo = np.zeros((u.shape[0], 3))
        pdf = np.zeros(u.shape[0])
        lib().orc_bsdf_sample(self.h, int(obj), _p(n, _f64p), _p(wi, _f64p), _p(u, _f64p), u.shape[0],
                              _p(wo, _f64p), _p(pdf, _f64p))
        return wo, pdf

    def chart(self, obj, xi):
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        out = np.zeros(12)
        on = lib().orc_chart(self.h, int(obj), _p(xi, _f64p), _p(out, _f64p))
        return bool(on), out[0:3], out[3:6], out[6:9], out[9:12]

    def newton(self, obj, xi, a_src, b_src, c_src, a_dst, b_dst, c_dst, dl0, tol, max_iter=5):
        v = [np.ascontiguousarray(x, dtype=np.float64) for x in (xi, a_src, b_src, a_dst, b_dst)]
        out = np.zeros(8)
        ok = lib().orc_newton(self.h, int(obj), _p(v[0], _f64p), _p(v[1], _f64p), _p(v[2], _f64p),
                              float(c_src), _p(v[3], _f64p), _p(v[4], _f64p), float(c_dst), float(dl0),
                              float(tol), int(max_iter), _p(out, _f64p))
        return dict(ok=bool(ok), xi=out[0:2].copy(), iters=int(out[2]), det_dxi=out[3],
                    det_area=out[4], F=out[5:7].copy(), status=int(out[7]))

    def vel_eval(self, obj, xi, a, va, b, vb, c=0.0):
        """Path-velocity constraint function of the reconnection vertex on
        object obj's chart in the loaded frame: (U, gradient[2], Hessian[2x2])."""
        v = [np.ascontiguousarray(x, dtype=np.float64) for x in (xi, a, va, b, vb)]
        out = np.zeros(6)
        ok = lib().orc_vel_eval(self.h, int(obj), *[_p(x, _f64p) for x in v], float(c), _p(out, _f64p))
        H = np.array([[out[3], out[4]], [out[4], out[5]]])
        return bool(ok), out[0], out[1:3].copy(), H
