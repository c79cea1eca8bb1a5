"""Pins of the oracle's materials and shadow rays.

* The BSDF sampler (cosine-weighted for Lambert; GGX half vectors drawn
  proportional to D(h) cos(theta_h), Walter et al. 2007) returns the density
  of the directions it draws: for every bin of solid angle Omega_b,
  E[1_b(w) / pdf(w)] = Omega_b exactly when pdf is that density, whatever the
  distribution.  A pdf missing its half-vector Jacobian 1/(4|w_i.h|) is off
  by a factor of up to four and fails.
* Importance-sampled directional albedo E[f cos / pdf] equals the albedo
  integrated by quadrature of the BSDF's own evaluation; the albedo is at most
  1 (energy conservation), equals rho for Lambert, tends to the Fresnel
  reflectance F0 as the roughness vanishes at normal incidence (the mirror
  limit of a microfacet model), and the BSDF is reciprocal.
* The any-hit query of the shadow rays agrees with the closest hit found by
  brute force: a segment of length t_max is blocked exactly when the closest
  hit lies before t_max.
"""
import math

import numpy as np
import pytest

from paper_2605_11536_amd import scenes


def _material_oracle(oracle_lib, mtype, albedo=0.0, alpha=0.0, f0=0.0):
    b = scenes._Builder()
    m = b.material(mtype, albedo=albedo, alpha=alpha, f0=f0)
    b.grid(scenes._quad((-1, -1, 0), (2, 0, 0), (0, 2, 0)), m)
    scene = b.build(np.stack([scenes._identity_xform()]))
    sensor = scenes.Sensor(width=4, height=4, temporal=0, spatial_rounds=0)
    return oracle_lib.Oracle(scene, sensor, num_threads=1)


def _incident(theta_deg):
    t = math.radians(theta_deg)
    return np.array([math.sin(t), 0.0, math.cos(t)])


N = np.array([0.0, 0.0, 1.0])


def _albedo_quadrature(o, wi, nb=2000, ng=96):
    """Integral of f(wi, wo) cos(theta_o) over the sphere, in polar
    coordinates about the mirror direction (dense near it: beta = pi s^2)."""
    r = 2.0 * wi[2] * N - wi
    t1 = np.cross(r, [0.0, 1.0, 0.0])
    if np.linalg.norm(t1) < 1e-6:
        t1 = np.cross(r, [1.0, 0.0, 0.0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(r, t1)
    s = (np.arange(nb) + 0.5) / nb
    beta = math.pi * s * s
    dbeta = 2.0 * math.pi * s / nb
    gam = (np.arange(ng) + 0.5) / ng * 2.0 * math.pi
    B, G = np.meshgrid(beta, gam, indexing="ij")
    wo = (np.cos(B)[..., None] * r + np.sin(B)[..., None] * (np.cos(G)[..., None] * t1 + np.sin(G)[..., None] * t2))
    wo = wo.reshape(-1, 3)
    f = o.bsdf(0, N, wi, wo)
    cos_o = np.maximum(wo[:, 2], 0.0)
    w = (np.sin(B) * dbeta[:, None] * (2.0 * math.pi / ng)).reshape(-1)
    return float(np.sum(f * cos_o * w))


CASES = [(scenes.MAT_LAMBERT, 0.7, 0.0, 0.0)] + [(scenes.MAT_GGX, 0.0, a, 0.8) for a in (0.05, 0.2, 0.5)]


@pytest.mark.parametrize("mat", CASES, ids=["lambert", "ggx0.05", "ggx0.2", "ggx0.5"])
@pytest.mark.parametrize("theta_i", [0.0, 45.0, 75.0])
def test_sampler_density_is_the_returned_pdf(oracle_lib, mat, theta_i):
    o = _material_oracle(oracle_lib, *mat)
    wi = _incident(theta_i)
    n = 400_000
    u = np.random.default_rng(7).random((n, 2))
    wo, pdf = o.bsdf_sample(0, N, wi, u)
    ok = pdf > 0
    assert ok.mean() > 0.5
    assert np.all(wo[ok, 2] > 0)                      # reflection only, above the surface
    nc, nphi = 16, 32
    ci = np.minimum((wo[:, 2] * nc).astype(int), nc - 1)
    phi = np.mod(np.arctan2(wo[:, 1], wo[:, 0]), 2 * math.pi)
    pi_ = np.minimum((phi / (2 * math.pi) * nphi).astype(int), nphi - 1)
    binid = np.where(ok, ci * nphi + pi_, -1)
    omega = (1.0 / nc) * (2 * math.pi / nphi)          # every bin's solid angle
    inv = np.where(ok, 1.0 / np.where(ok, pdf, 1.0), 0.0)
    zs = []
    for b in range(nc * nphi):
        sel = binid == b
        if sel.sum() < 200:
            continue
        x = np.where(sel, inv, 0.0)
        est, se = x.mean(), x.std(ddof=1) / math.sqrt(n)
        zs.append((est - omega) / se)
    zs = np.array(zs)
    assert zs.size >= 4
    assert np.max(np.abs(zs)) < 5.0, zs
    assert np.mean(zs * zs) < 2.0, np.mean(zs * zs)
    o.close()


@pytest.mark.parametrize("mat", CASES, ids=["lambert", "ggx0.05", "ggx0.2", "ggx0.5"])
@pytest.mark.parametrize("theta_i", [0.0, 45.0, 75.0])
def test_sampled_albedo_matches_quadrature_and_conserves_energy(oracle_lib, mat, theta_i):
    o = _material_oracle(oracle_lib, *mat)
    wi = _incident(theta_i)
    n = 400_000
    u = np.random.default_rng(11).random((n, 2))
    wo, pdf = o.bsdf_sample(0, N, wi, u)
    ok = pdf > 0
    f = o.bsdf(0, N, wi, wo)
    x = np.where(ok, f * np.maximum(wo[:, 2], 0.0) / np.where(ok, pdf, 1.0), 0.0)
    a_is, se = x.mean(), x.std(ddof=1) / math.sqrt(n)
    a_q = _albedo_quadrature(o, wi)
    assert abs(a_is - a_q) <= 4 * se + 2e-3 * a_q, (a_is, a_q, se)
    assert a_q <= 1.0 + 1e-3
    if mat[0] == scenes.MAT_LAMBERT:
        assert a_q == pytest.approx(mat[1], rel=1e-3)
        assert np.allclose(f[ok], mat[1] / math.pi)
    o.close()


def test_ggx_mirror_limit_and_reciprocity(oracle_lib):
    # near-mirror at normal incidence: the albedo is the Fresnel reflectance F0
    for f0 in (0.8, 1.0):
        o = _material_oracle(oracle_lib, scenes.MAT_GGX, alpha=0.02, f0=f0)
        a = _albedo_quadrature(o, _incident(0.0), nb=4000)
        assert a == pytest.approx(f0, rel=5e-3), (f0, a)
        o.close()
    # energy: even with F0 = 1 a rough surface reflects no more than it receives
    o = _material_oracle(oracle_lib, scenes.MAT_GGX, alpha=0.5, f0=1.0)
    for th in (0.0, 60.0, 85.0):
        assert _albedo_quadrature(o, _incident(th)) <= 1.0
    o.close()
    # reciprocity f(wi, wo) = f(wo, wi) on random pairs of the upper hemisphere
    rng = np.random.default_rng(3)
    for alpha in (0.05, 0.3):
        o = _material_oracle(oracle_lib, scenes.MAT_GGX, alpha=alpha, f0=0.8)
        d = rng.normal(size=(200, 2, 3))
        d[..., 2] = np.abs(d[..., 2])
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        for a, b in d:
            fab = o.bsdf(0, N, a, b[None])[0]
            fba = o.bsdf(0, N, b, a[None])[0]
            assert fab == pytest.approx(fba, rel=1e-9, abs=1e-300)
        o.close()


def _segments(rng, n, lo, hi):
    o = rng.uniform(lo, hi, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


@pytest.mark.parametrize("which", ["box", "glossy", "nlos"])
def test_any_hit_matches_brute_force_closest_hit(oracle_lib, which):
    if which == "glossy":
        w = scenes.glossy_dynamic(width=8, height=8, frames=2, ground_cells=40, sphere_nu=16, sphere_nv=10)
        lo, hi, tmax = [-5, -0.5, -5], [5, 2, 5], 6.0
    elif which == "nlos":
        w = scenes.nlos_confocal(scan=8, frames=2, torus_nu=60, torus_nv=24)
        lo, hi, tmax = [-1, -1, 0.05], [1, 1, 1.5], 2.0
    else:
        w = scenes.cornell_box(width=8, height=8)
        lo, hi, tmax = [-0.95] * 3, [0.95] * 3, 2.0
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    o.load_frame(w.frames[-1])
    rng = np.random.default_rng(5)
    org, dirs = _segments(rng, 3000, lo, hi)
    lens = rng.uniform(0.0, tmax, size=3000)
    blocked = free = 0
    for a, d, L in zip(org, dirs, lens):
        prim, r = o.trace(a, d, brute=True)
        t = r[0] if prim >= 0 else math.inf
        if abs(t - L) < 1e-9 * max(1.0, L):
            continue                                   # a hit at the segment's end: either answer is right
        expect = t < L
        assert o.occluded(a, d, L) == expect, (a, d, L, t)
        blocked += expect
        free += not expect
    assert blocked > 300 and free > 300, (blocked, free)
    o.close()
