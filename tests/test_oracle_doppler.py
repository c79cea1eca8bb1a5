"""Pins of the oracle's Doppler domain (Sec. 4.6): planes over the path
velocity u = -dl/dt (eq. optical_path_velocity) and the shift under the
path-velocity constraint.

* u of a reconnection vertex's two segments equals minus the time derivative
  of their length, taken as a central difference over the scene moved rigidly
  (objects, endpoints) by +-eps: this fixes the sign convention, the rigid
  motion of chart points and the vertex velocities independently of the
  formula the oracle evaluates.
* Its chart gradient and Hessian (derived here; the supplement that holds
  them is not available) against finite differences over the chart, on a
  translating quad and on a spinning sphere (curvature terms).
* Closed-form Doppler spectrum of a receding Lambertian plane under a
  co-located camera and light: with the plane at depth d receding at speed s,
  a point seen at angle theta has u = -2 s cos(theta) and path length
  l = -4 s d / u, so the plane transient's closed form
  sum_q I_q a_p = (4 rho I / d)(1/l_lo - 1/l_hi) becomes rho I du / (s d^2)
  for every velocity bin of width du whose ring lies in the field of view (a
  flat spectrum); the same for a camera and light approaching the plane
  (u = +2 s cos(theta)), which pins the endpoint velocities.
* Unbiasedness of ToF ReSTIR in the velocity domain against plain path
  tracing (GRIS is unbiased for any bijective shift, Sec. 3.2.3).
"""
import math

import numpy as np
import pytest

from paper_2605_11536_amd import scenes


def _rodrigues(w, t):
    """Rotation by the angle |w| t about w (numpy, independent of the oracle)."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w) * t
    if th == 0.0:
        return np.eye(3)
    k = w / np.linalg.norm(w)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * (K @ K)


def _moved_frame(fr, t):
    """The frame with every object advanced by its rigid motion over time t."""
    xf = fr.xforms.astype(np.float64).reshape(-1, 3, 4).copy()
    for o in range(xf.shape[0]):
        v, w = fr.velocities[o, :3].astype(np.float64), fr.velocities[o, 3:].astype(np.float64)
        xf[o, :, :3] = _rodrigues(w, t) @ xf[o, :, :3]
        xf[o, :, 3] = xf[o, :, 3] + v * t
    out = scenes.Frame(**{f.name: getattr(fr, f.name) for f in scenes.dataclasses.fields(fr)})
    out.xforms = xf.reshape(-1, 12).astype(np.float32)
    return out


def _cases(w):
    sc = w.scene
    big = 5          # first face of the receding box (translation only)
    sph = sc.num_objects - 1   # spinning sphere
    a, va = np.array([0.1, 0.2, 0.9]), np.array([0.3, -0.2, 0.5])
    b, vb = np.array([-0.8, 0.6, -0.9]), np.array([0.0, 0.0, 0.0])
    return [(big, np.array([0.4, 0.6]), a, va, b, vb), (big, np.array([0.25, 0.3]), b, vb, a, va),
            (sph, np.array([0.35, 0.4]), a, va, b, vb), (sph, np.array([0.7, 0.55]), a, vb, b, va)]


def test_path_velocity_is_minus_time_derivative_of_length(oracle_lib):
    w = scenes.doppler_boxes(width=8, height=8, frames=1)
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    fr = w.frames[0]
    eps = 2e-3
    for obj, xi, a, va, b, vb in _cases(w):
        o.load_frame(fr)
        ok, U, g, H = o.vel_eval(obj, xi, a, va, b, vb)
        assert ok
        lens = []
        for t in (eps, -eps):
            o.load_frame(_moved_frame(fr, t))
            on, p, *_ = o.chart(obj, xi)
            at, bt = a + va * t, b + vb * t
            lens.append(np.linalg.norm(p - at) + np.linalg.norm(p - bt))
        u_fd = -(lens[0] - lens[1]) / (2 * eps)
        assert abs(U) > 0.05          # a case with motion
        assert U == pytest.approx(u_fd, abs=2e-3 * max(1.0, abs(U))), (obj, xi, U, u_fd)
    o.close()


def test_path_velocity_chart_derivatives_match_finite_differences(oracle_lib):
    w = scenes.doppler_boxes(width=8, height=8, frames=1)
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    o.load_frame(w.frames[0])
    h = 1e-5
    for obj, xi, a, va, b, vb in _cases(w):
        ok, U, g, H = o.vel_eval(obj, xi, a, va, b, vb, c=0.3)
        assert ok
        gfd = np.zeros(2)
        Hfd = np.zeros((2, 2))
        for k in range(2):
            e = np.zeros(2)
            e[k] = h
            _, Up, gp, _ = o.vel_eval(obj, xi + e, a, va, b, vb, c=0.3)
            _, Um, gm, _ = o.vel_eval(obj, xi - e, a, va, b, vb, c=0.3)
            gfd[k] = (Up - Um) / (2 * h)
            Hfd[:, k] = (gp - gm) / (2 * h)
        scale = max(1.0, np.abs(g).max())
        assert np.allclose(g, gfd, atol=1e-6 * scale), (obj, g, gfd)
        hs = max(1.0, np.abs(H).max())
        assert np.allclose(H, Hfd, atol=1e-5 * hs), (obj, H, Hfd)
        assert H[0, 1] == H[1, 0]
    # a static configuration has no path velocity and a vanishing gradient
    z = np.zeros(3)
    ok, U, g, H = o.vel_eval(0, np.array([0.3, 0.4]), np.array([0.1, 0.2, 0.9]), z, np.array([0.5, 0.5, 0.5]), z)
    assert ok and U == 0.0 and np.all(g == 0.0) and np.all(H == 0.0)
    o.close()


@pytest.mark.parametrize("mover", ["plane", "camera_and_light"])
def test_receding_plane_doppler_spectrum_closed_form(oracle_lib, mover):
    d, rho, I, s = 1.0, 0.5, 1.0, 1.0
    nb, du = 10, 0.025
    sign = -1.0 if mover == "plane" else 1.0
    t0 = -2.0 if mover == "plane" else 1.75
    gc = -1.9 if mover == "plane" else 1.9
    w = scenes.lambert_plane(depth=d, albedo=rho, intensity=I, width=256, height=256, fov=60.0,
                             n_bins=nb, bin_t0=t0, bin_width=du, gate_enabled=1, gate_center=gc,
                             gate_width=0.05, domain=scenes.DOMAIN_VELOCITY)
    fr = w.frames[0]
    if mover == "plane":
        fr.velocities = np.array([[0.0, 0.0, -s, 0.0, 0.0, 0.0]], dtype=np.float32)
    else:
        fr.velocities = np.zeros((1, 6), dtype=np.float32)
        fr.cam_vel = (0.0, 0.0, -s)
        fr.light_vel = (0.0, 0.0, -s)
    o = oracle_lib.Oracle(w.scene, w.sensor)
    tan_half = math.tan(math.radians(30.0))
    a_p = (2 * tan_half / 256) ** 2
    sums, gates = [], []
    for f in range(12):
        fr.index = f
        out = o.render(fr)
        sums.append(out["pt_hist"].sum(axis=(1, 2)) * a_p * du)
        gates.append(out["pt_image"].sum() * a_p * 0.05)
    sums = np.array(sums)
    exp = rho * I * du / (s * d * d)
    mean = sums.mean(0)
    se = sums.std(0, ddof=1) / math.sqrt(len(sums)) + 1e-12
    assert np.all(np.abs(mean - exp) < 4.5 * se + 1e-3 * exp), (mean / exp)
    assert np.mean(gates) == pytest.approx(rho * I * 0.05 / (s * d * d), rel=5e-3)
    # the sign: nothing lands on the other side of zero
    w2 = scenes.lambert_plane(depth=d, albedo=rho, intensity=I, width=64, height=64, fov=60.0,
                              n_bins=2, bin_t0=-3.0, bin_width=3.0, gate_enabled=0,
                              domain=scenes.DOMAIN_VELOCITY)
    o2 = oracle_lib.Oracle(w2.scene, w2.sensor)
    h = o2.render(fr)["pt_hist"].sum(axis=(1, 2))
    assert (h[0] > 0 and h[1] == 0) if sign < 0 else (h[0] == 0 and h[1] > 0)
    o.close()
    o2.close()


def test_velocity_domain_rejects_length_only_shifts(oracle_lib):
    w = scenes.doppler_boxes(width=8, height=8, frames=1, bin_radius=1)
    with pytest.raises(Exception):
        oracle_lib.Oracle(w.scene, w.sensor)


def _doppler_unbiased(oracle_lib, seeds, frames, **kw):
    r_img, p_img, r_h, p_h = [], [], [], []
    conv = 0
    for seed in range(seeds):
        w = scenes.doppler_boxes(width=24, height=24, frames=frames, seed=seed, spatial_radius=4, **kw)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        pts, pth = [], []
        for fr in w.frames:
            out = o.render(fr)
            pts.append(out["pt_image"])
            pth.append(out["pt_hist"])
        conv += o.stats()["newton_converged"]
        r_img.append(out["image"])
        r_h.append(out["hist"])
        p_img.append(np.mean(pts, 0))
        p_h.append(np.mean(pth, 0))
        o.close()
    return np.array(r_img), np.array(p_img), np.array(r_h), np.array(p_h), conv


@pytest.mark.parametrize("temporal", [0, 1])
def test_doppler_restir_unbiased_against_plain_pt(oracle_lib, temporal):
    n = 64
    R, Pt, Rh, Ph, conv = _doppler_unbiased(oracle_lib, n, 2 if temporal else 1, temporal=temporal)
    assert conv > 0   # the path-velocity Newton solve runs and converges
    for r, p in ((R.sum(axis=(1, 2)), Pt.sum(axis=(1, 2))),
                 (Rh.sum(axis=(2, 3))[:, 1:6].sum(1), Ph.sum(axis=(2, 3))[:, 1:6].sum(1))):
        z = (r.mean() - p.mean()) / math.sqrt(r.var(ddof=1) / n + p.var(ddof=1) / n)
        assert abs(z) < 3.5, z
    # per bin, over the sensor
    rb, pb = Rh.sum(axis=(2, 3)), Ph.sum(axis=(2, 3))
    vr, vp = rb.var(0, ddof=1) / n, pb.var(0, ddof=1) / n
    mask = (vr > 0) & (vp > 0)
    assert mask.sum() >= 4
    zb = (rb.mean(0) - pb.mean(0))[mask] / np.sqrt(vr + vp)[mask]
    assert np.all(np.abs(zb) < 4.0), zb
