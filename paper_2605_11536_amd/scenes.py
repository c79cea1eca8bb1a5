"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *describes* scenes: object-local geometry, materials,
per-frame rigid transforms, camera/light poses and the sensor settings.  It
holds none of the method's arithmetic (no path lengths, shading, sampling or
resampling), so it may feed both the HIP path and the CPU oracle.

Every float array is float32; the oracle promotes the same float32 values to
float64, so both sides start from bit-identical inputs.

Object model (shared vocabulary of the two sides, defined here as data):

* GRID object: an (nu+1) x (nv+1) lattice of object-local vertices
  ``V[j*(nu+1) + i]`` (i along u, j along v).  Cell (i, j) is split into
  triangle A = (V[i,j], V[i+1,j], V[i,j+1]) and triangle B =
  (V[i+1,j+1], V[i,j+1], V[i+1,j]).  ``wrap_u``/``wrap_v`` mark periodic
  directions (the last column/row then repeats the first).  The surface chart
  is xi = (u, v) in cell units.
* SPHERE object: analytic sphere (local centre, radius) with the chart
  xi = (theta, phi) about the object's local z axis.

Per-frame object transforms are rigid, stored row-major as 3x4 ``[R | t]``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

OBJ_GRID = 0
OBJ_SPHERE = 1
MAT_LAMBERT = 0
MAT_GGX = 1
CAM_PINHOLE = 0
CAM_ORTHO = 1
LIGHT_POINT = 0
LIGHT_CONFOCAL = 1
SHIFT_NAIVE = 0
SHIFT_PATHLEN = 1
STAGE_FINAL = 2
STAGE_TEMPORAL = 1
STAGE_CANONICAL = 0
DOMAIN_TIME = 0
DOMAIN_VELOCITY = 1
MIS_GBH = 0
MIS_PAIRWISE = 1

f32 = np.float32


@dataclasses.dataclass
class Scene:
    """Objects, materials and object-local vertices (all float32/int32)."""

    obj_type: np.ndarray        # int32 [O]
    obj_material: np.ndarray    # int32 [O]
    obj_grid: np.ndarray        # int32 [O, 5]: nu, nv, wrap_u, wrap_v, vertex_offset
    obj_sphere: np.ndarray      # float32 [O, 4]: local centre xyz, radius
    mat_type: np.ndarray        # int32 [Mt]
    mat_params: np.ndarray      # float32 [Mt, 3]: albedo, alpha, f0
    vertices: np.ndarray        # float32 [V, 3]
    scene_scale: float          # s_c = bbox diagonal / sqrt(3) at frame 0

    @property
    def num_objects(self) -> int:
        return int(self.obj_type.shape[0])

    @property
    def num_triangles(self) -> int:
        g = self.obj_grid
        return int(sum(2 * g[o, 0] * g[o, 1] for o in range(self.num_objects)
                       if self.obj_type[o] == OBJ_GRID))


@dataclasses.dataclass
class Sensor:
    """Sensor, time-domain and reuse settings (one per render stream)."""

    width: int
    height: int
    full_width: int = 0          # 0 -> same as width (no crop)
    full_height: int = 0
    crop_x0: int = 0
    crop_y0: int = 0
    camera_model: int = CAM_PINHOLE
    light_model: int = LIGHT_POINT
    light_intensity: float = 1.0
    count_camera_leg: int = 1
    jitter: int = 1
    gate_enabled: int = 1
    gate_center: float = 3.0
    gate_width: float = 0.05
    n_bins: int = 0
    bin_t0: float = 0.0
    bin_width: float = 0.1
    n_min: int = 2
    n_max: int = 2
    m_init: int = 1
    temporal: int = 1
    spatial_rounds: int = 1
    spatial_k: int = 5
    spatial_radius: int = 10
    m_cap: float = 20.0
    newton_tol_rel: float = 0.01   # tolerance = newton_tol_rel * gate/bin width
    newton_max_iter: int = 5
    j_max: float = 100.0
    shift_mode: int = SHIFT_PATHLEN
    include_direct: int = 0
    debug_stage: int = STAGE_FINAL
    bin_radius: int = 0            # bin-axis reuse: bins b +- 1..bin_radius (0 = off)
    shrink_k: float = 1.0          # shrink mapping of initial gate samples: rough gate K x wider (1 = off)
    shrink_r: float = 1.0          # fraction of the path trees sampled from the wide gate (R < 1: MIS with the gate)
    domain: int = DOMAIN_TIME      # planes over path length (time) or path velocity (Doppler)
    round_trip: int = 1            # keep a Newton shift only if its inverse returns to the source vertex
    mis_mode: int = MIS_GBH        # spatial reuse weights: generalized balance heuristic or pairwise
    seed: int = 0

    def __post_init__(self):
        if self.full_width == 0:
            self.full_width = self.width
        if self.full_height == 0:
            self.full_height = self.height

    @property
    def b_tot(self) -> int:
        return self.n_bins + (1 if self.gate_enabled else 0)


@dataclasses.dataclass
class Frame:
    """Per-frame poses: camera, light and the rigid object transforms."""

    index: int
    cam_pos: np.ndarray          # float32 [3]
    cam_fwd: np.ndarray          # float32 [3]
    cam_up: np.ndarray           # float32 [3]
    fov_y_deg: float             # pinhole vertical field of view
    ortho_half: np.ndarray       # float32 [2]: ortho half extents (x, y)
    light_pos: np.ndarray        # float32 [3]
    xforms: np.ndarray           # float32 [O, 12]
    # instantaneous velocities (the Doppler domain): per object linear v and
    # angular w (a point x moves at v + w x (x - t), t the object's origin),
    # camera and light velocities; None / zero = at rest
    velocities: Optional[np.ndarray] = None   # float32 [O, 6]
    cam_vel: tuple = (0.0, 0.0, 0.0)
    light_vel: tuple = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    sensor: Sensor
    frames: List[Frame]


# --------------------------------------------------------------------------
# small helpers (geometry construction only)
# --------------------------------------------------------------------------

def _identity_xform() -> np.ndarray:
    return np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=f32)


def _xform(rot: np.ndarray, trans) -> np.ndarray:
    m = np.zeros((3, 4), dtype=np.float64)
    m[:, :3] = rot
    m[:, 3] = trans
    return m.reshape(12).astype(f32)


def _rot_axis_angle(axis, deg: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    th = math.radians(deg)
    c, s = math.cos(th), math.sin(th)
    x, y, z = a
    return np.array([
        [c + x * x * (1 - c), x * y * (1 - c) - z * s, x * z * (1 - c) + y * s],
        [y * x * (1 - c) + z * s, c + y * y * (1 - c), y * z * (1 - c) - x * s],
        [z * x * (1 - c) - y * s, z * y * (1 - c) + x * s, c + z * z * (1 - c)],
    ])


class _Builder:
    def __init__(self):
        self.types, self.mats, self.grids, self.spheres = [], [], [], []
        self.verts: list = []
        self.nverts = 0
        self.mat_type, self.mat_params = [], []

    def material(self, mtype: int, albedo=0.0, alpha=0.0, f0=0.0) -> int:
        self.mat_type.append(mtype)
        self.mat_params.append((albedo, alpha, f0))
        return len(self.mat_type) - 1

    def grid(self, lattice: np.ndarray, mat: int, wrap_u=0, wrap_v=0) -> int:
        """lattice: float [nv+1, nu+1, 3] of object-local vertices."""
        nvp, nup, _ = lattice.shape
        self.types.append(OBJ_GRID)
        self.mats.append(mat)
        self.grids.append((nup - 1, nvp - 1, wrap_u, wrap_v, self.nverts))
        self.spheres.append((0, 0, 0, 0))
        flat = lattice.reshape(-1, 3)
        self.verts.append(flat)
        self.nverts += flat.shape[0]
        return len(self.types) - 1

    def sphere(self, centre, radius, mat: int) -> int:
        self.types.append(OBJ_SPHERE)
        self.mats.append(mat)
        self.grids.append((0, 0, 0, 0, 0))
        self.spheres.append((*centre, radius))
        return len(self.types) - 1

    def build(self, xforms0: np.ndarray) -> Scene:
        verts = (np.concatenate(self.verts, 0) if self.verts
                 else np.zeros((0, 3))).astype(f32)
        scene = Scene(
            obj_type=np.array(self.types, dtype=np.int32),
            obj_material=np.array(self.mats, dtype=np.int32),
            obj_grid=np.array(self.grids, dtype=np.int32).reshape(-1, 5),
            obj_sphere=np.array(self.spheres, dtype=f32).reshape(-1, 4),
            mat_type=np.array(self.mat_type, dtype=np.int32),
            mat_params=np.array(self.mat_params, dtype=f32).reshape(-1, 3),
            vertices=verts,
            scene_scale=0.0,
        )
        scene.scene_scale = float(f32(_scene_scale(scene, xforms0)))
        return scene


def _scene_scale(scene: Scene, xforms: np.ndarray) -> float:
    """Bounding-box diagonal / sqrt(3) of the world-space scene at frame 0."""
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    for o in range(scene.num_objects):
        m = xforms[o].astype(np.float64).reshape(3, 4)
        if scene.obj_type[o] == OBJ_GRID:
            nu, nv, _, _, off = scene.obj_grid[o]
            v = scene.vertices[off: off + (nu + 1) * (nv + 1)].astype(np.float64)
            w = v @ m[:, :3].T + m[:, 3]
            lo = np.minimum(lo, w.min(0))
            hi = np.maximum(hi, w.max(0))
        else:
            c = scene.obj_sphere[o, :3].astype(np.float64)
            r = float(scene.obj_sphere[o, 3])
            cw = m[:, :3] @ c + m[:, 3]
            lo = np.minimum(lo, cw - r)
            hi = np.maximum(hi, cw + r)
    return float(np.linalg.norm(hi - lo) / math.sqrt(3.0))


def _quad(p0, pu, pv) -> np.ndarray:
    """1x1 grid lattice for the parallelogram p0 + a*pu + b*pv."""
    p0, pu, pv = (np.asarray(x, dtype=np.float64) for x in (p0, pu, pv))
    lat = np.zeros((2, 2, 3))
    lat[0, 0] = p0
    lat[0, 1] = p0 + pu
    lat[1, 0] = p0 + pv
    lat[1, 1] = p0 + pu + pv
    return lat


def _latlong_sphere(radius: float, nu: int, nv: int) -> np.ndarray:
    """(nv+1) x (nu+1) latitude/longitude lattice, poles on the local z axis."""
    lat = np.zeros((nv + 1, nu + 1, 3))
    for j in range(nv + 1):
        th = math.pi * j / nv
        for i in range(nu + 1):
            ph = 2.0 * math.pi * (i % nu) / nu
            lat[j, i] = (radius * math.sin(th) * math.cos(ph),
                         radius * math.sin(th) * math.sin(ph),
                         radius * math.cos(th))
    lat[0, :] = (0.0, 0.0, radius)
    lat[nv, :] = (0.0, 0.0, -radius)
    return lat


def _value_noise_2d(x: np.ndarray, y: np.ndarray, seed: int, period=None) -> np.ndarray:
    """Smooth lattice value noise in [-1, 1] (hashing integer lattice points)."""
    rng = np.random.default_rng(seed)
    table = rng.uniform(-1.0, 1.0, size=4096)
    perm = rng.permutation(4096)

    def h(ix, iy):
        if period is not None:
            ix = np.mod(ix, period[0])
            iy = np.mod(iy, period[1])
        return table[perm[(perm[np.mod(ix, 4096)] + iy) % 4096]]

    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx = x - x0
    fy = y - y0
    sx = fx * fx * (3 - 2 * fx)
    sy = fy * fy * (3 - 2 * fy)
    a = h(x0, y0) * (1 - sx) + h(x0 + 1, y0) * sx
    b = h(x0, y0 + 1) * (1 - sx) + h(x0 + 1, y0 + 1) * sx
    return a * (1 - sy) + b * sy


def _fbm(x, y, seed, octaves=4, period=None):
    tot = np.zeros_like(x)
    amp, freq, norm = 1.0, 1.0, 0.0
    for o in range(octaves):
        per = None if period is None else (period[0] * int(freq), period[1] * int(freq))
        tot += amp * _value_noise_2d(x * freq, y * freq, seed + 17 * o, per)
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return tot / norm


def _pinhole_frame(index, cam_pos, look_at, up, fov, light_pos, xforms) -> Frame:
    cam_pos = np.asarray(cam_pos, dtype=np.float64)
    fwd = np.asarray(look_at, dtype=np.float64) - cam_pos
    fwd /= np.linalg.norm(fwd)
    return Frame(index=index, cam_pos=cam_pos.astype(f32), cam_fwd=fwd.astype(f32),
                 cam_up=np.asarray(up, dtype=f32), fov_y_deg=float(fov),
                 ortho_half=np.zeros(2, dtype=f32),
                 light_pos=np.asarray(light_pos, dtype=f32),
                 xforms=np.ascontiguousarray(xforms, dtype=f32))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def cornell_box(width=64, height=64, frames=4, seed=0, **sensor_kw) -> Workload:
    """Tiny plain-method scene: open box of 5 Lambertian quads + one sphere.

    Box [-1,1]^3 open at z=+1, albedo 0.7; sphere r=0.3 at (0,-0.7,-0.3),
    albedo 0.5 (chart poles on the world x axis); pinhole camera and a
    co-located isotropic point light at (0,0,1) looking down -z, 90 deg FOV.
    Max 2 bounces, gate of width 0.05 centred at path length 3.0, static.
    """
    b = _Builder()
    wall = b.material(MAT_LAMBERT, albedo=0.7)
    ball = b.material(MAT_LAMBERT, albedo=0.5)
    b.grid(_quad((-1, -1, -1), (2, 0, 0), (0, 2, 0)), wall)   # back
    b.grid(_quad((-1, -1, -1), (0, 0, 2), (2, 0, 0)), wall)   # floor
    b.grid(_quad((-1, 1, -1), (2, 0, 0), (0, 0, 2)), wall)    # ceiling
    b.grid(_quad((-1, -1, -1), (0, 2, 0), (0, 0, 2)), wall)   # left
    b.grid(_quad((1, -1, -1), (0, 0, 2), (0, 2, 0)), wall)    # right
    b.sphere((0.0, 0.0, 0.0), 0.3, ball)
    nobj = 6
    xf = np.stack([_identity_xform()] * nobj)
    # sphere: chart pole axis (local z) mapped to world x, centre (0,-0.7,-0.3)
    rot = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], dtype=np.float64)
    xf[5] = _xform(rot, (0.0, -0.7, -0.3))
    scene = b.build(xf)
    kw = dict(width=width, height=height, gate_center=3.0, gate_width=0.05,
              n_min=2, n_max=2, m_init=1, temporal=1, spatial_rounds=1,
              spatial_k=5, spatial_radius=10, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    fr = [_pinhole_frame(f, (0, 0, 1), (0, 0, 0), (0, 1, 0), 90.0, (0, 0, 1), xf)
          for f in range(frames)]
    return Workload("cornell_box_64", scene, sensor, fr)


def glossy_box(width=32, height=32, frames=3, seed=0, wall_alpha=0.3, floor_alpha=0.12, ball_alpha=0.25,
               move=1.0, **sensor_kw) -> Workload:
    """The tiny box with GGX surfaces on both sides of the reconnection
    roughness 0.2 and a moving sphere: back, ceiling and side walls GGX with
    wall_alpha and the sphere with ball_alpha (rough: reconnectable), the
    floor with floor_alpha (smooth: replayed), F0 0.8; the sphere moves
    +0.05 move in x and turns 5 move degrees about the vertical per frame."""
    b = _Builder()
    wall = b.material(MAT_GGX, alpha=wall_alpha, f0=0.8)
    floor = b.material(MAT_GGX, alpha=floor_alpha, f0=0.8)
    ball = b.material(MAT_GGX, alpha=ball_alpha, f0=0.8)
    b.grid(_quad((-1, -1, -1), (2, 0, 0), (0, 2, 0)), wall)    # back
    b.grid(_quad((-1, -1, -1), (0, 0, 2), (2, 0, 0)), floor)   # floor
    b.grid(_quad((-1, 1, -1), (2, 0, 0), (0, 0, 2)), wall)     # ceiling
    b.grid(_quad((-1, -1, -1), (0, 2, 0), (0, 0, 2)), wall)    # left
    b.grid(_quad((1, -1, -1), (0, 0, 2), (0, 2, 0)), wall)     # right
    b.sphere((0.0, 0.0, 0.0), 0.3, ball)
    base = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], dtype=np.float64)

    def xforms_at(f):
        xf = np.stack([_identity_xform()] * 6)
        xf[5] = _xform(_rot_axis_angle((0, 1, 0), 5.0 * move * f) @ base, (-0.1 + 0.05 * move * f, -0.7, -0.3))
        return xf

    scene = b.build(xforms_at(0))
    kw = dict(width=width, height=height, gate_center=4.0, gate_width=0.4, n_min=2, n_max=3, m_init=1,
              temporal=1, spatial_rounds=1, spatial_k=5, spatial_radius=4, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    fr = [_pinhole_frame(f, (0, 0, 1), (0, 0, 0), (0, 1, 0), 90.0, (0, 0, 1), xforms_at(f)) for f in range(frames)]
    return Workload("glossy_box", scene, sensor, fr)


def lambert_plane(depth=1.0, albedo=0.5, intensity=1.0, width=64, height=64,
                  fov=60.0, half_size=50.0, **sensor_kw) -> Workload:
    """A single Lambertian plane z=-depth facing a pinhole at the origin with
    a co-located isotropic point light (direct illumination only)."""
    b = _Builder()
    m = b.material(MAT_LAMBERT, albedo=albedo)
    h = half_size
    b.grid(_quad((-h, -h, -depth), (2 * h, 0, 0), (0, 2 * h, 0)), m)
    xf = np.stack([_identity_xform()])
    scene = b.build(xf)
    kw = dict(width=width, height=height, n_min=1, n_max=1, include_direct=1,
              light_intensity=intensity, temporal=0, spatial_rounds=0)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    fr = [_pinhole_frame(0, (0, 0, 0), (0, 0, -1), (0, 1, 0), fov, (0, 0, 0), xf)]
    return Workload("lambert_plane", scene, sensor, fr)


def glossy_dynamic(width=512, height=512, frames=60, seed=0, ground_cells=160,
                   sphere_nu=64, sphere_nv=40, n_spheres=8, **sensor_kw) -> Workload:
    """Dynamic glossy scene, ~92k triangles.

    Ground: 160x160-cell lattice over [-5,5]^2 displaced by 0.15*fbm (4-octave
    value noise), Lambertian albedo 0.5.  Eight latitude/longitude spheres of
    64x40 cells (5,120 triangles each), radius U[0.4,0.8], GGX with alpha
    U[0.05,0.5] and F0 0.8; each translates 0.02 per frame in a random
    horizontal direction and rotates 1 degree per frame about a random axis.
    Camera (0,2.5,7.5) looking at (0,0.5,0), 40 deg FOV, co-located light.
    Max 3 bounces; 256-bin histogram (t0=12, width 0.1) plus a gate at 17.0 of
    width 0.1; temporal reuse plus one spatial round (k=5, radius 30 px).
    """
    rng = np.random.default_rng(1000 + seed)
    b = _Builder()
    ground_mat = b.material(MAT_LAMBERT, albedo=0.5)
    n = ground_cells
    xs = np.linspace(-5.0, 5.0, n + 1)
    zs = np.linspace(-5.0, 5.0, n + 1)
    X, Z = np.meshgrid(xs, zs)            # [v, u]
    Y = 0.15 * _fbm(X * 0.8, Z * 0.8, seed=7 + seed)
    lat = np.stack([X, Y, Z], -1)
    # orient so the geometric normal (J_u x J_v) points up: u along +z? use u=x, v=z
    # J_u x J_v = (+x) x (+z) = -y, so flip the v direction
    lat = lat[::-1].copy()
    b.grid(lat, ground_mat)
    centres, radii = [], []
    tries = 0
    while len(centres) < n_spheres and tries < 10000:
        tries += 1
        r = rng.uniform(0.4, 0.8)
        c = np.array([rng.uniform(-3.2, 3.2), 0.0, rng.uniform(-3.2, 2.5)])
        if any(np.linalg.norm(c[[0, 2]] - c2[[0, 2]]) < r + r2 + 0.3
               for c2, r2 in zip(centres, radii)):
            continue
        c[1] = r + 0.2
        centres.append(c)
        radii.append(r)
    sph_objs = []
    for s in range(n_spheres):
        alpha = rng.uniform(0.05, 0.5)
        m = b.material(MAT_GGX, alpha=alpha, f0=0.8)
        sph_objs.append(b.grid(_latlong_sphere(radii[s], sphere_nu, sphere_nv), m, wrap_u=1))
    vel = []
    axes = []
    for s in range(n_spheres):
        a = rng.uniform(0, 2 * math.pi)
        vel.append(np.array([math.cos(a), 0.0, math.sin(a)]) * 0.02)
        ax = rng.normal(size=3)
        axes.append(ax / np.linalg.norm(ax))
    nobj = 1 + n_spheres

    def xforms_at(f):
        xf = np.stack([_identity_xform()] * nobj)
        for s in range(n_spheres):
            rot = _rot_axis_angle(axes[s], 1.0 * f)
            xf[1 + s] = _xform(rot, centres[s] + f * vel[s])
        return xf

    scene = b.build(xforms_at(0))
    kw = dict(width=width, height=height, gate_enabled=1, gate_center=17.0,
              gate_width=0.1, n_bins=256, bin_t0=12.0, bin_width=0.1, n_min=2,
              n_max=3, m_init=1, temporal=1, spatial_rounds=1, spatial_k=5,
              spatial_radius=30, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    fr = [_pinhole_frame(f, (0, 2.5, 7.5), (0, 0.5, 0), (0, 1, 0), 40.0,
                         (0, 2.5, 7.5), xforms_at(f)) for f in range(frames)]
    return Workload(f"glossy_dynamic_{width}", scene, sensor, fr)


def _catmull_rom(points: np.ndarray, t: float) -> np.ndarray:
    """Closed Catmull-Rom spline through `points` at parameter t in [0, 1)."""
    n = len(points)
    x = (t % 1.0) * n
    i = int(math.floor(x))
    u = x - i
    p0, p1, p2, p3 = (points[(i + k) % n] for k in (-1, 0, 1, 2))
    return 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u
                  + (-p0 + 3 * p1 - 3 * p2 + p3) * u * u * u)


def specular_stress(width=1920, height=1080, frames=120, seed=0, ground_cells=480, n_spheres=32, sphere_nu=96,
                    sphere_nv=80, n_specular=19, **sensor_kw) -> Workload:
    """Near-specular stress scene, about 0.95M triangles.

    Ground: 480x480-cell lattice over [-8,8]^2 displaced by 0.2*fbm, Lambertian
    albedo 0.5 (461k triangles).  32 latitude/longitude spheres of 96x80 cells
    (15,360 triangles each), radius U[0.3,0.7], resting on the ground: the
    first 19 GGX with alpha 0.01 and F0 0.8 (30.7% of the triangles), the
    others Lambertian with albedo U[0.3,0.8].  Static geometry; the camera
    (with a co-located light) follows a closed Catmull-Rom spline through six
    points around the scene at heights 2-4, looking at (0,0.5,0), 50 deg FOV,
    one turn over `frames` frames.  Up to 4 bounces; 512-bin histogram
    (t0=10, width 0.05) plus a gate at 20.0 of width 0.1; temporal reuse plus
    one spatial round (k=5, radius 30 px).
    """
    rng = np.random.default_rng(5000 + seed)
    b = _Builder()
    ground_mat = b.material(MAT_LAMBERT, albedo=0.5)
    n = ground_cells
    xs = np.linspace(-8.0, 8.0, n + 1)
    X, Z = np.meshgrid(xs, xs)
    Y = 0.2 * _fbm(X * 0.6, Z * 0.6, seed=17 + seed)
    lat = np.stack([X, Y, Z], -1)[::-1].copy()   # normal up
    b.grid(lat, ground_mat)
    centres, radii = [], []
    tries = 0
    while len(centres) < n_spheres and tries < 20000:
        tries += 1
        r = rng.uniform(0.3, 0.7)
        c = np.array([rng.uniform(-6.0, 6.0), 0.0, rng.uniform(-6.0, 6.0)])
        if np.hypot(c[0], c[2]) > 6.5 or any(np.linalg.norm(c[[0, 2]] - c2[[0, 2]]) < r + r2 + 0.2
                                              for c2, r2 in zip(centres, radii)):
            continue
        c[1] = r + 0.25
        centres.append(c)
        radii.append(r)
    sphere_lat = {}
    for k in range(len(centres)):
        if k < n_specular:
            m = b.material(MAT_GGX, alpha=0.01, f0=0.8)
        else:
            m = b.material(MAT_LAMBERT, albedo=float(rng.uniform(0.3, 0.8)))
        key = round(radii[k], 6)
        if key not in sphere_lat:
            sphere_lat[key] = _latlong_sphere(radii[k], sphere_nu, sphere_nv)
        b.grid(sphere_lat[key], m, wrap_u=1)
    nobj = 1 + len(centres)
    xf = np.stack([_identity_xform()] * nobj)
    for k in range(len(centres)):
        xf[1 + k] = _xform(np.eye(3), centres[k])
    scene = b.build(xf)
    kw = dict(width=width, height=height, gate_enabled=1, gate_center=20.0, gate_width=0.1, n_bins=512,
              bin_t0=10.0, bin_width=0.05, n_min=2, n_max=4, m_init=1, temporal=1, spatial_rounds=1,
              spatial_k=5, spatial_radius=30, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    ang = np.linspace(0.0, 2 * math.pi, 6, endpoint=False)
    ctrl = np.stack([np.array([9.0 * math.cos(a), 3.0 + math.sin(2 * a), 9.0 * math.sin(a)]) for a in ang])
    fr = []
    for f in range(frames):
        cp = _catmull_rom(ctrl, f / max(frames, 1))
        fr.append(_pinhole_frame(f, cp, (0, 0.5, 0), (0, 1, 0), 50.0, cp, xf))
    return Workload(f"specular_stress_{width}x{height}", scene, sensor, fr)


def nlos_confocal(scan=64, frames=32, seed=0, torus_nu=250, torus_nv=100,
                  n_bins=1024, **sensor_kw) -> Workload:
    """NLOS time-resolved simulation: relay wall + hidden displaced torus.

    Relay wall z=0, 2x2 units, Lambertian 0.8, scanned confocally on a 64x64
    grid over [-0.9,0.9]^2 (orthographic scan sensor, laser spot at the scan
    point, time origin at the wall).  Hidden torus R=0.35, r=0.12, 250x100
    cells (50k triangles), displaced 0.02*noise along its normal, centre
    (0,0,1), albedo 0.5; it moves +0.005 in x and rotates 1 degree about y per
    frame.  1024 bins of width 0.004 from t0=0; only wall-hidden-wall paths.
    """
    b = _Builder()
    wall_m = b.material(MAT_LAMBERT, albedo=0.8)
    tor_m = b.material(MAT_LAMBERT, albedo=0.5)
    b.grid(_quad((-1, -1, 0), (2, 0, 0), (0, 2, 0)), wall_m)
    R, r = 0.35, 0.12
    us = np.arange(torus_nu + 1) / torus_nu * 2 * math.pi
    vs = np.arange(torus_nv + 1) / torus_nv * 2 * math.pi
    U, V = np.meshgrid(us, vs)                       # [v, u]
    disp = 0.02 * _fbm(U / (2 * math.pi) * 12.0, V / (2 * math.pi) * 6.0, seed=31 + seed,
                       period=(12, 6))
    rr = r + disp
    X = (R + rr * np.cos(V)) * np.cos(U)
    Y = (R + rr * np.cos(V)) * np.sin(U)
    Z = rr * np.sin(V)
    lat = np.stack([X, Y, Z], -1)
    lat[:, torus_nu] = lat[:, 0]
    lat[torus_nv, :] = lat[0, :]
    b.grid(lat, tor_m, wrap_u=1, wrap_v=1)

    def xforms_at(f):
        xf = np.stack([_identity_xform()] * 2)
        rot = _rot_axis_angle((0, 1, 0), 1.0 * f)
        xf[1] = _xform(rot, (0.005 * f, 0.0, 1.0))
        return xf

    scene = b.build(xforms_at(0))
    kw = dict(width=scan, height=scan, camera_model=CAM_ORTHO, light_model=LIGHT_CONFOCAL,
              count_camera_leg=0, jitter=0, gate_enabled=0, n_bins=n_bins, bin_t0=0.0,
              bin_width=0.004, n_min=2, n_max=2, m_init=1, temporal=1,
              spatial_rounds=1, spatial_k=5, spatial_radius=4, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    half = 0.9 * scan / (scan - 1)
    fr = []
    for f in range(frames):
        fr.append(Frame(index=f, cam_pos=np.array([0, 0, 0.5], dtype=f32),
                        cam_fwd=np.array([0, 0, -1], dtype=f32),
                        cam_up=np.array([0, 1, 0], dtype=f32), fov_y_deg=0.0,
                        ortho_half=np.array([half, half], dtype=f32),
                        light_pos=np.zeros(3, dtype=f32), xforms=xforms_at(f)))
    return Workload(f"nlos_confocal_{scan}", scene, sensor, fr)


def nlos_plane(depth=1.0, wall_albedo=0.8, albedo=0.5, intensity=1.0, scan=32, frames=1, seed=0,
               half_size=5.0, **sensor_kw) -> Workload:
    """Confocal scan of the relay wall z=0 (2x2, as in nlos_confocal) with a
    large Lambertian plane z=depth facing it in place of the hidden object:
    every scan point sees the same wall-plane-wall transient, which has a
    closed form."""
    b = _Builder()
    wall_m = b.material(MAT_LAMBERT, albedo=wall_albedo)
    hid_m = b.material(MAT_LAMBERT, albedo=albedo)
    b.grid(_quad((-1, -1, 0), (2, 0, 0), (0, 2, 0)), wall_m)
    h = half_size
    b.grid(_quad((-h, -h, depth), (0, 2 * h, 0), (2 * h, 0, 0)), hid_m)
    xf = np.stack([_identity_xform()] * 2)
    scene = b.build(xf)
    kw = dict(width=scan, height=scan, camera_model=CAM_ORTHO, light_model=LIGHT_CONFOCAL,
              count_camera_leg=0, jitter=0, gate_enabled=0, n_bins=8, bin_t0=2.0 * depth,
              bin_width=0.1 * depth, n_min=2, n_max=2, m_init=1, light_intensity=intensity, temporal=1,
              spatial_rounds=1, spatial_k=5, spatial_radius=4, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    half = 0.9 * scan / (scan - 1)
    fr = [Frame(index=f, cam_pos=np.array([0, 0, 0.5 * depth], dtype=f32), cam_fwd=np.array([0, 0, -1], dtype=f32),
                cam_up=np.array([0, 1, 0], dtype=f32), fov_y_deg=0.0, ortho_half=np.array([half, half], dtype=f32),
                light_pos=np.zeros(3, dtype=f32), xforms=xf) for f in range(frames)]
    return Workload(f"nlos_plane_{scan}", scene, sensor, fr)


def lambert_sphere_interior(radius=1.0, albedo=0.5, intensity=1.0, width=32, height=32,
                           frames=1, seed=0, **sensor_kw) -> Workload:
    """Inside an analytic Lambertian sphere, pinhole camera and isotropic point
    light at its centre.  Every pixel sees the same transient, which has a
    closed form per bounce count."""
    b = _Builder()
    m = b.material(MAT_LAMBERT, albedo=albedo)
    b.sphere((0.0, 0.0, 0.0), radius, m)
    xf = np.stack([_identity_xform()])
    scene = b.build(xf)
    kw = dict(width=width, height=height, n_min=2, n_max=2, light_intensity=intensity,
              gate_enabled=1, gate_center=3.5 * radius, gate_width=0.1 * radius, n_bins=20,
              bin_t0=2.0 * radius, bin_width=0.1 * radius, temporal=1, spatial_rounds=1,
              spatial_k=3, spatial_radius=4, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    fr = [_pinhole_frame(f, (0, 0, 0), (0, 0, -1), (0, 1, 0), 60.0, (0, 0, 0), xf)
          for f in range(frames)]
    return Workload("lambert_sphere_interior", scene, sensor, fr)


def _box_faces(b: "_Builder", h, mat) -> List[int]:
    """Six quads of the axis-aligned box [-h, h] (object-local), one object each."""
    hx, hy, hz = h
    faces = [((-hx, -hy, -hz), (2 * hx, 0, 0), (0, 2 * hy, 0)),
             ((-hx, -hy, hz), (0, 2 * hy, 0), (2 * hx, 0, 0)),
             ((-hx, -hy, -hz), (0, 0, 2 * hz), (2 * hx, 0, 0)),
             ((-hx, hy, -hz), (2 * hx, 0, 0), (0, 0, 2 * hz)),
             ((-hx, -hy, -hz), (0, 2 * hy, 0), (0, 0, 2 * hz)),
             ((hx, -hy, -hz), (0, 0, 2 * hz), (0, 2 * hy, 0))]
    return [b.grid(_quad(*f), mat) for f in faces]


def doppler_boxes(width=64, height=64, frames=2, seed=0, dt=1.0 / 30.0, **sensor_kw) -> Workload:
    """Doppler scene (Sec. 4.6 and its evaluation): an open Lambertian room
    [-1,1]^3, a large box receding from the camera at 1 m/s, a small box
    approaching it at 1.5 m/s and a sphere spinning at 3 rad/s about the
    vertical axis; pinhole camera and co-located point light at (0,0,1)
    looking down -z.  The planes are 16 bins of 0.25 m/s over the path
    velocity u in [-2.0625, 1.9375) (u = 0, every static path, mid-bin) and a
    gate [-1.125, -0.875) on the receding box; spatial reuse only, as in the
    paper's Doppler demo.  Frames advance the motion by dt."""
    b = _Builder()
    wall = b.material(MAT_LAMBERT, albedo=0.7)
    big_m = b.material(MAT_LAMBERT, albedo=0.6)
    small_m = b.material(MAT_LAMBERT, albedo=0.5)
    ball = b.material(MAT_LAMBERT, albedo=0.5)
    b.grid(_quad((-1, -1, -1), (2, 0, 0), (0, 2, 0)), wall)   # back
    b.grid(_quad((-1, -1, -1), (0, 0, 2), (2, 0, 0)), wall)   # floor
    b.grid(_quad((-1, 1, -1), (2, 0, 0), (0, 0, 2)), wall)    # ceiling
    b.grid(_quad((-1, -1, -1), (0, 2, 0), (0, 0, 2)), wall)   # left
    b.grid(_quad((1, -1, -1), (0, 0, 2), (0, 2, 0)), wall)    # right
    big = _box_faces(b, (0.35, 0.3, 0.3), big_m)
    small = _box_faces(b, (0.18, 0.18, 0.18), small_m)
    sph = b.sphere((0.0, 0.0, 0.0), 0.25, ball)
    nobj = sph + 1
    big_c, big_v = np.array([-0.4, -0.7, -0.35]), np.array([0.0, 0.0, -1.0])
    small_c, small_v = np.array([0.45, -0.82, -0.25]), np.array([0.0, 0.0, 1.5])
    sph_c, sph_w = np.array([0.35, 0.35, -0.5]), np.array([0.0, 3.0, 0.0])
    # sphere chart poles on the world x axis, as in the Cornell box
    pole = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], dtype=np.float64)

    def poses(t):
        xf = np.stack([_identity_xform()] * nobj)
        for o in big:
            xf[o] = _xform(np.eye(3), big_c + big_v * t)
        for o in small:
            xf[o] = _xform(np.eye(3), small_c + small_v * t)
        ang = math.degrees(float(np.linalg.norm(sph_w)) * t)
        xf[sph] = _xform(_rot_axis_angle(sph_w, ang) @ pole, sph_c)
        return xf

    vel = np.zeros((nobj, 6), dtype=f32)
    vel[big, 0:3] = big_v
    vel[small, 0:3] = small_v
    vel[sph, 3:6] = sph_w
    scene = b.build(poses(0.0))
    kw = dict(width=width, height=height, domain=DOMAIN_VELOCITY, gate_enabled=1, gate_center=-1.0,
              gate_width=0.25, n_bins=16, bin_t0=-2.0625, bin_width=0.25, n_min=2, n_max=2, m_init=1,
              temporal=0, spatial_rounds=1, spatial_k=5, spatial_radius=10, seed=seed)
    kw.update(sensor_kw)
    sensor = Sensor(**kw)
    fr = []
    for f in range(frames):
        F = _pinhole_frame(f, (0, 0, 1), (0, 0, 0), (0, 1, 0), 90.0, (0, 0, 1), poses(f * dt))
        F.velocities = vel.copy()
        fr.append(F)
    return Workload("doppler_boxes", scene, sensor, fr)


WORKLOADS = {
    "lambert_sphere_interior": lambert_sphere_interior,
    "cornell_box": cornell_box,
    "glossy_dynamic": glossy_dynamic,
    "nlos_confocal": nlos_confocal,
    "lambert_plane": lambert_plane,
    "doppler_boxes": doppler_boxes,
}
