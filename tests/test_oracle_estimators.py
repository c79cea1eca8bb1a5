"""Statistical pins of the oracle's estimators.

* Closed-form transient of a Lambertian plane under a co-located point light
  (direct light; derived from the ToF path integral, Sec. 3.1): summed over
  the image plane, sum_q I_q a_p = (4 rho I / d)(1/l_lo - 1/l_hi) for a bin
  [l_lo, l_hi) whose ring lies inside the field of view.
* Closed-form 2- and 3-bounce transients inside a Lambertian sphere with the
  camera and light at its centre: between two points of a sphere
  cos*cos/r^2 = 1/(4R^2), so the chord length c has density c/(2R^2) on
  [0, 2R] and h_2(l) = rho^2 I/(pi R^2) * (l-2R)/(2R^2); h_3 is the
  convolution of two chord densities times rho^3 I/(pi R^2).
* Unbiasedness of ToF ReSTIR (GRIS is unbiased, Sec. 3.2.3): its per-pixel
  mean over independent seeds equals plain path tracing's, including with
  Newton forced to fail and with the naive (non path-length-aware) shift.
"""
import math

import numpy as np
import pytest

from paper_2605_11536_amd import scenes


def _chord_pdf(c, R):
    return np.where((c >= 0) & (c <= 2 * R), c / (2 * R * R), 0.0)


def test_plane_transient_closed_form(oracle_lib):
    d, rho, I = 1.0, 0.5, 1.0
    nb, t0, bw = 12, 2.0, 0.025
    w = scenes.lambert_plane(depth=d, albedo=rho, intensity=I, width=256, height=256, fov=60.0,
                             n_bins=nb, bin_t0=t0, bin_width=bw, gate_enabled=1,
                             gate_center=2.1, gate_width=0.05)
    o = oracle_lib.Oracle(w.scene, w.sensor)
    tan_half = math.tan(math.radians(30.0))
    a_p = (2 * tan_half / 256) ** 2
    sums = []
    gates = []
    for f in range(20):
        fr = w.frames[0]
        fr.index = f
        out = o.render(fr)
        sums.append(out["pt_hist"].sum(axis=(1, 2)) * a_p * bw)
        gates.append(out["pt_image"].sum() * a_p * 0.05)
    sums = np.array(sums)
    lo = t0 + bw * np.arange(nb)
    hi = lo + bw
    exp = 4 * rho * I / d * (1 / lo - 1 / hi)
    mean = sums.mean(0)
    se = sums.std(0, ddof=1) / math.sqrt(len(sums)) + 1e-12
    assert np.all(np.abs(mean - exp) < 4.5 * se), (mean / exp)
    assert np.mean(gates) == pytest.approx(4 * rho * I / d * (1 / 2.075 - 1 / 2.125), rel=5e-3)
    # ReSTIR with only the deterministic direct term equals plain PT exactly
    assert np.allclose(out["hist"], out["pt_hist"])


def _sphere_expect(rho, I, R, lo, hi, bounces):
    """Bin-averaged closed-form transient inside the sphere."""
    out = []
    for a, b in zip(lo, hi):
        ls = np.linspace(a, b, 401)
        if bounces == 2:
            h = rho ** 2 * I / (math.pi * R * R) * _chord_pdf(ls - 2 * R, R)
        else:
            cs = np.linspace(0, 2 * R, 4001)
            h = []
            for l in ls:
                s = l - 2 * R
                h.append(np.trapezoid(_chord_pdf(cs, R) * _chord_pdf(s - cs, R), cs))
            h = rho ** 3 * I / (math.pi * R * R) * np.array(h)
        out.append(np.trapezoid(h, ls) / (b - a))
    return np.array(out)


@pytest.mark.parametrize("bounces", [2, 3])
def test_sphere_interior_closed_form_plain_pt(oracle_lib, bounces):
    R, rho, I = 1.0, 0.5, 1.0
    nb = 20 if bounces == 2 else 40
    w = scenes.lambert_sphere_interior(radius=R, albedo=rho, intensity=I, width=32, height=32,
                                       n_min=bounces, n_max=bounces, n_bins=nb, bin_width=0.1,
                                       temporal=0, spatial_rounds=0)
    o = oracle_lib.Oracle(w.scene, w.sensor)
    per = []
    for f in range(24):
        fr = w.frames[0]
        fr.index = f
        per.append(o.render(fr)["pt_hist"].mean(axis=(1, 2)))
    per = np.array(per)
    lo = 2 * R + 0.1 * np.arange(nb)
    exp = _sphere_expect(rho, I, R, lo, lo + 0.1, bounces)
    mean, se = per.mean(0), per.std(0, ddof=1) / math.sqrt(len(per))
    assert np.all(np.abs(mean - exp) < 4.5 * se + 1e-3 * exp.max()), (mean - exp) / (se + 1e-15)
    assert abs(mean.sum() - exp.sum()) < 4 * math.sqrt((se ** 2).sum())


@pytest.mark.parametrize("mis", [scenes.MIS_GBH, scenes.MIS_PAIRWISE], ids=["gbh", "pairwise"])
def test_sphere_interior_closed_form_restir(oracle_lib, mis):
    """ReSTIR (temporal + spatial, path-length-aware shift on the curved
    sphere chart) matches the closed form in expectation over seeds, with
    the generalized balance heuristic and with pairwise MIS in the spatial
    pass."""
    R, rho, I = 1.0, 0.5, 1.0
    nb = 20
    lo = 2 * R + 0.1 * np.arange(nb)
    exp = _sphere_expect(rho, I, R, lo, lo + 0.1, 2)
    per = []
    for seed in range(16):
        w = scenes.lambert_sphere_interior(radius=R, albedo=rho, intensity=I, width=24, height=24,
                                           n_bins=nb, frames=3, seed=seed, mis_mode=mis)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        for fr in w.frames:
            out = o.render(fr)
        per.append(out["hist"].mean(axis=(1, 2)))
        o.close()
    per = np.array(per)
    mean, se = per.mean(0), per.std(0, ddof=1) / math.sqrt(len(per))
    assert np.all(np.abs(mean - exp) < 4.5 * se + 1e-3 * exp.max()), (mean - exp) / (se + 1e-15)
    assert abs(mean.sum() - exp.sum()) < 4 * math.sqrt((se ** 2).sum())


def _unbiased_case(oracle_lib, seeds, scene=scenes.cornell_box, last_frame_pt=False, **kw):
    """Per seed, ReSTIR's last frame and plain PT, the gate image and the
    histogram bins flattened into one row of (plane, pixel) entries.  Static
    scenes average plain PT over the frames; in a moving scene plain PT of the
    last frame alone estimates what the last ReSTIR frame estimates."""
    r_all, p_all = [], []
    for seed in range(seeds):
        if scene is scenes.cornell_box:
            w = scene(width=64, height=64, frames=3, seed=seed, gate_width=0.2, spatial_radius=4, n_bins=16,
                      bin_t0=2.6, bin_width=0.1, **kw)
        else:
            w = scene(width=96, height=96, frames=3, seed=seed, **kw)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        outs = [o.render(fr) for fr in w.frames]
        o.close()
        flat = lambda d, a, b: np.concatenate([d[a].ravel()] + ([d[b].ravel()] if b in d else []))
        r_all.append(flat(outs[-1], "image", "hist"))
        pts = [flat(d, "pt_image", "pt_hist") for d in outs]
        p_all.append(pts[-1] if last_frame_pt else np.mean(pts, 0))
    return np.array(r_all), np.array(p_all)


def _assert_unbiased(R, Pt, min_entries=500):
    """Seeds are independent.  The sensor sums agree within 3 sigma.  Per
    (plane, pixel) entry, z of the difference of the means is near normal where
    both sides are non-zero in at least an eighth of the seeds (rarer paths
    make plain PT's mean and variance skewed); there at most 0.5% of the
    entries have |z| > 3."""
    n = R.shape[0]
    rs, ps = R.sum(axis=1), Pt.sum(axis=1)
    z_sum = (rs.mean() - ps.mean()) / math.sqrt(rs.var(ddof=1) / n + ps.var(ddof=1) / n)
    mr, mp = R.mean(0), Pt.mean(0)
    vr, vp = R.var(0, ddof=1) / n, Pt.var(0, ddof=1) / n
    mask = ((R != 0).sum(0) >= n // 8) & ((Pt != 0).sum(0) >= n // 8)
    z = (mr - mp)[mask] / np.sqrt(vr + vp)[mask]
    frac = float(np.mean(np.abs(z) > 3.0))
    print(f"sensor-sum z {z_sum:+.2f}; {mask.sum()} entries, {frac * 100:.2f}% with |z| > 3, mean z {z.mean():+.3f}")
    assert abs(z_sum) < 3.0, z_sum
    assert mask.sum() > min_entries, mask.sum()
    assert frac <= 0.005, frac


@pytest.mark.parametrize("variant", ["pathlen", "newton_fails", "naive", "pairwise"])
def test_restir_unbiased_against_plain_pt(oracle_lib, variant):
    kw = {}
    if variant == "newton_fails":
        kw = dict(newton_max_iter=0)
    elif variant == "naive":
        kw = dict(shift_mode=scenes.SHIFT_NAIVE)
    elif variant == "pairwise":
        kw = dict(mis_mode=scenes.MIS_PAIRWISE)
    R, Pt = _unbiased_case(oracle_lib, 256, **kw)
    _assert_unbiased(R, Pt)


def test_restir_unbiased_glossy_moving_scene(oracle_lib):
    """A box of GGX surfaces on both sides of the reconnection roughness with
    a moving, turning GGX sphere: the temporal history is re-evaluated in the
    new frame (suffix positions, throughput and visibility), and ReSTIR's last
    frame matches plain PT of that frame.  Narrow GGX lobes lit by a point
    light make the per-pixel estimates heavy-tailed (a per-pixel z of plain PT
    against itself at 16x the samples has |z| > 3 on 16% of the pixels), so
    the comparison is on 6x6-pixel block sums against plain PT with 16 path
    trees per pixel, with plain PT at one tree as the control of the same
    statistic."""
    n, res, bs = 256, 48, 6

    def blocks(img):
        return img.reshape(res // bs, bs, res // bs, bs).sum(axis=(1, 3)).ravel()

    R, P, Q = [], [], []
    for seed in range(n):
        w = scenes.glossy_box(width=res, height=res, frames=3, seed=seed)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        outs = [o.render(fr) for fr in w.frames]
        o.close()
        R.append(blocks(outs[-1]["image"]))
        P.append(blocks(outs[-1]["pt_image"]))
        wq = scenes.glossy_box(width=res, height=res, frames=3, seed=10_000 + seed, m_init=16, temporal=0,
                               spatial_rounds=0)
        o = oracle_lib.Oracle(wq.scene, wq.sensor)
        Q.append(blocks([o.render(fr) for fr in wq.frames][-1]["pt_image"]))
        o.close()
    R, P, Q = np.array(R), np.array(P), np.array(Q)

    def zs(A):
        va, vq = A.var(0, ddof=1) / n, Q.var(0, ddof=1) / n
        m = (va + vq) > 0
        return (A.mean(0) - Q.mean(0))[m] / np.sqrt(va + vq)[m]

    zr, zp = zs(R), zs(P)
    rs, qs = R.sum(1), Q.sum(1)
    z_sum = (rs.mean() - qs.mean()) / math.sqrt(rs.var(ddof=1) / n + qs.var(ddof=1) / n)
    print(f"sensor-sum z {z_sum:+.2f}; {zr.size} blocks: ReSTIR max |z| {np.abs(zr).max():.2f} mean z "
          f"{zr.mean():+.3f}; plain PT max |z| {np.abs(zp).max():.2f} mean z {zp.mean():+.3f}")
    assert zr.size >= 40
    assert abs(z_sum) < 3.0
    assert np.sum(np.abs(zr) > 3.0) <= 1 and np.abs(zr).max() < 4.0
    assert abs(zr.mean()) < 0.5


def _gate_sweep(oracle_lib, seed, step, frames=3, **kw):
    w = scenes.cornell_box(width=32, height=32, frames=frames, seed=seed, gate_width=0.2, spatial_radius=4, **kw)
    o = oracle_lib.Oracle(w.scene, w.sensor)
    c0 = w.sensor.gate_center
    for f, fr in enumerate(w.frames):
        if f:
            o.set_gate_center(c0 + step * f)
        out = o.render(fr)
    st = o.stats()
    o.close()
    return out, st


def test_gate_shift_temporal_reuse_lands_in_the_moved_gate(oracle_lib):
    """Time-gate shifting (Sec. 4.1): with the gate moved by +0.1 per frame
    (width 0.2) and temporal reuse only, previous-frame paths shifted by
    Delta l = +0.1 land in the new gate.  Shifting by the opposite amount puts
    every one of them outside it (checked once by mutating the sign: 0 of 53
    succeed), so a wrong sign or a dropped Delta l fails this bound."""
    ok = att = 0
    for seed in range(3):
        _, st = _gate_sweep(oracle_lib, seed, 0.1, spatial_rounds=0)
        ok += st["shifts_ok"]
        att += st["newton_attempts"]
    assert att > 50
    assert ok / att > 0.3, (ok, att)


def test_restir_unbiased_with_gate_sweep(oracle_lib):
    """ReSTIR with the gate moving between frames (temporal reuse with
    Delta l = the gate's move, plus spatial reuse) matches plain PT at the
    final gate in expectation over seeds."""
    n = 96
    r, p = [], []
    for seed in range(n):
        out, _ = _gate_sweep(oracle_lib, seed, 0.05)
        r.append(out["image"].sum())
        p.append(out["pt_image"].sum())
    r, p = np.array(r), np.array(p)
    z = (r.mean() - p.mean()) / math.sqrt(r.var(ddof=1) / n + p.var(ddof=1) / n)
    assert abs(z) < 3.5, z


def test_bin_reuse_shifts_land_in_the_target_bin(oracle_lib):
    """Bin-axis reuse (Sec. 4.5) alone: a sample of bin b' enters bin b with
    Delta l = (b - b') * bin width.  Most such shifts land in the target bin
    on the sphere interior (smooth chart, every length reachable); with the
    sign of Delta l flipped the target is 2 |b - b'| bins away and none do,
    so a wrong sign or a dropped Delta l fails this bound."""
    w = scenes.lambert_sphere_interior(radius=1.0, albedo=0.5, intensity=1.0, width=16, height=16, n_bins=20,
                                       frames=1, temporal=0, spatial_rounds=0, bin_radius=1)
    o = oracle_lib.Oracle(w.scene, w.sensor)
    o.render(w.frames[0])
    st = o.stats()
    o.close()
    assert st["newton_attempts"] > 500
    assert st["shifts_ok"] / st["newton_attempts"] > 0.5, st


@pytest.mark.parametrize("radius", [1, 2])
def test_sphere_interior_closed_form_restir_bin_reuse(oracle_lib, radius):
    """ReSTIR with bin-axis reuse (plus temporal and spatial reuse) matches the
    closed-form transient inside the sphere in expectation over seeds."""
    R, rho, I = 1.0, 0.5, 1.0
    nb = 20
    lo = 2 * R + 0.1 * np.arange(nb)
    exp = _sphere_expect(rho, I, R, lo, lo + 0.1, 2)
    per = []
    for seed in range(16):
        w = scenes.lambert_sphere_interior(radius=R, albedo=rho, intensity=I, width=24, height=24,
                                           n_bins=nb, frames=3, seed=seed, bin_radius=radius)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        for fr in w.frames:
            out = o.render(fr)
        per.append(out["hist"].mean(axis=(1, 2)))
        o.close()
    per = np.array(per)
    mean, se = per.mean(0), per.std(0, ddof=1) / math.sqrt(len(per))
    assert np.all(np.abs(mean - exp) < 4.5 * se + 1e-3 * exp.max()), (mean - exp) / (se + 1e-15)
    assert abs(mean.sum() - exp.sum()) < 4 * math.sqrt((se ** 2).sum())


def test_restir_unbiased_with_bin_reuse(oracle_lib):
    """Box scene, 16 bins over the gate's neighbourhood, bin-axis reuse with
    temporal and spatial reuse: the histogram matches plain PT in expectation
    over seeds (sensor sum per bin)."""
    n = 64
    r, p = [], []
    for seed in range(n):
        w = scenes.cornell_box(width=24, height=24, frames=3, seed=seed, gate_width=0.2, spatial_radius=4,
                               n_bins=16, bin_t0=2.6, bin_width=0.1, bin_radius=2)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        pts = []
        for fr in w.frames:
            out = o.render(fr)
            pts.append(out["pt_hist"].sum(axis=(1, 2)))
        r.append(out["hist"].sum(axis=(1, 2)))
        p.append(np.mean(pts, 0))
        o.close()
    r, p = np.array(r), np.array(p)
    tot_r, tot_p = r.sum(1), p.sum(1)
    z = (tot_r.mean() - tot_p.mean()) / math.sqrt(tot_r.var(ddof=1) / n + tot_p.var(ddof=1) / n)
    assert abs(z) < 3.5, z
    vr, vp = r.var(0, ddof=1) / n, p.var(0, ddof=1) / n
    zb = (r.mean(0) - p.mean(0)) / np.sqrt(vr + vp + 1e-30)
    assert np.all(np.abs(zb[(vr > 0) & (vp > 0)]) < 4.0), zb


@pytest.mark.parametrize("reuse", [False, True])
def test_shrink_mapping_sphere_closed_form(oracle_lib, reuse):
    """Shrink mapping (Sec. 4.4.2), all samples in a gate K = 5 times wider:
    inside the sphere every rough-gate length maps onto the gate and nearly
    every shrink succeeds, so the gate image matches the gate's closed form
    in expectation (a dropped 1/K is off by a factor K, a wrong Delta l moves
    the samples out of the gate)."""
    R, rho, I = 1.0, 0.5, 1.0
    kw = {} if reuse else dict(temporal=0, spatial_rounds=0)
    exp = float(_sphere_expect(rho, I, R, [3.45], [3.55], 2)[0])
    per = []
    for seed in range(24):
        w = scenes.lambert_sphere_interior(radius=R, albedo=rho, intensity=I, width=24, height=24, n_bins=0,
                                           frames=2, seed=seed, shrink_k=5.0, **kw)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        for fr in w.frames:
            out = o.render(fr)
        per.append(out["image"].mean())
        st = o.stats()
        o.close()
        if not reuse:   # every shift is a shrink (a third of the pixels hold a rough-gate sample); nearly all succeed
            assert st["shifts"] > 0.25 * 24 * 24 * 2 and st["shifts_ok"] > 0.95 * st["shifts"], st
    per = np.array(per)
    mean, se = per.mean(), per.std(ddof=1) / math.sqrt(len(per))
    assert abs(mean - exp) < 4 * se + 2e-3 * exp, ((mean - exp) / se, mean, exp)


def _shrink_r_sums(oracle_lib, r, seeds, **kw):
    rs, ps = [], []
    for seed in range(seeds):
        w = scenes.cornell_box(width=32, height=32, frames=1, seed=seed, gate_width=0.05, m_init=3, shrink_k=20.0,
                               shrink_r=r, temporal=0, spatial_rounds=0, **kw)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        out = o.render(w.frames[0])
        rs.append(out["image"].sum())
        ps.append(out["pt_image"].sum())
        o.close()
    return np.array(rs), np.array(ps)


def test_shrink_mapping_with_canonical_samples_is_unbiased(oracle_lib):
    """Shrink mapping with R < 1 (Sec. 4.4.2): of three path trees per pixel
    two sample the gate and one a gate K = 20 times wider whose winner is
    shrunk; GRIS with the generalized balance heuristic over the two
    techniques (confidences 2 and 1) is unbiased, while R = 1 (all trees in
    the wide gate) is biased dark where shrinks fail, as the paper notes."""
    n = 96
    rs, ps = _shrink_r_sums(oracle_lib, 1.0 / 3.0, n)
    z = (rs.mean() - ps.mean()) / math.sqrt(rs.var(ddof=1) / n + ps.var(ddof=1) / n)
    assert abs(z) < 3.5, (z, rs.mean(), ps.mean())
    r1, p1 = _shrink_r_sums(oracle_lib, 1.0, n)
    z1 = (r1.mean() - p1.mean()) / math.sqrt(r1.var(ddof=1) / n + p1.var(ddof=1) / n)
    assert z1 < -4.0, z1   # the R = 1 bias this test would miss if it had no power



def test_shrink_mapping_with_canonical_samples_identity_is_exact(oracle_lib):
    """Under the naive shift no path is moved: a wide-gate sample enters the
    gate by the identity when it lies there, and the balance weights of the
    two techniques are their confidences, 2/3 (two gate trees) and 1/3 (one
    wide tree).  With one candidate per tree (n = 2 only) and no reuse the
    merged estimate then equals plain path tracing exactly, per seed (equal
    weights would lose a sixth)."""
    rs, ps = [], []
    for seed in range(16):
        w = scenes.cornell_box(width=32, height=32, frames=1, seed=seed, gate_width=0.2, m_init=3, shrink_k=5.0,
                               shrink_r=1.0 / 3.0, temporal=0, spatial_rounds=0, shift_mode=scenes.SHIFT_NAIVE)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        out = o.render(w.frames[0])
        rs.append(out["image"])
        ps.append(out["pt_image"])
        o.close()
    assert np.sum(ps) > 0
    assert np.allclose(np.array(rs), np.array(ps), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("reuse", [False, True])
def test_shrink_mapping_with_canonical_samples_sphere_closed_form(oracle_lib, reuse):
    """R = 1/2 (one of two path trees per pixel in a gate K = 5 times wider)
    inside the sphere: the gate image matches the gate's closed form in
    expectation, alone and followed by temporal and spatial reuse."""
    R, rho, I = 1.0, 0.5, 1.0
    kw = {} if reuse else dict(temporal=0, spatial_rounds=0)
    exp = float(_sphere_expect(rho, I, R, [3.45], [3.55], 2)[0])
    per = []
    for seed in range(24):
        w = scenes.lambert_sphere_interior(radius=R, albedo=rho, intensity=I, width=24, height=24, n_bins=0,
                                           frames=2, seed=seed, shrink_k=5.0, shrink_r=0.5, m_init=2, **kw)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        for fr in w.frames:
            out = o.render(fr)
        per.append(out["image"].mean())
        o.close()
    per = np.array(per)
    mean, se = per.mean(), per.std(ddof=1) / math.sqrt(len(per))
    assert abs(mean - exp) < 4 * se + 2e-3 * exp, ((mean - exp) / se, mean, exp)


def _confocal_plane_bins(depth, rho_w, rho_h, power, lo, hi):
    """Wall-plane-wall transient of a confocal scan point (Sec. 5 "Light
    Source": the laser spot on the wall re-emits as a Lambertian point, the
    time origin is at the wall): a Lambertian plane at depth D parallel to the
    wall gives, per unit path length over [l_lo, l_hi),
    P rho_w^2 rho_h D^4 / (3 pi^2) ((l_lo/2)^-6 - (l_hi/2)^-6) / (l_hi - l_lo).
    (Integrand (rho_w/pi) cos_g (rho_h/pi) cos_h P (rho_w/pi) cos_g / r^2 in
    the solid angle at the spot, cos_g = cos_h = D/r, over the plane:
    2 pi D^4 int r^-7 dr.)"""
    rl, rh = lo / 2.0, hi / 2.0
    return power * rho_w ** 2 * rho_h * depth ** 4 / (3 * math.pi ** 2) * (rl ** -6 - rh ** -6) / (hi - lo)


def test_confocal_plane_transient_closed_form(oracle_lib):
    D, rw, rh, P = 1.0, 0.8, 0.5, 2.0
    w = scenes.nlos_plane(depth=D, wall_albedo=rw, albedo=rh, intensity=P, scan=32, frames=96, temporal=0,
                          spatial_rounds=0)
    o = oracle_lib.Oracle(w.scene, w.sensor)
    per = []
    for fr in w.frames:
        per.append(o.render(fr)["pt_hist"])
    o.close()
    per = np.array(per).reshape(len(w.frames), w.sensor.n_bins, -1)      # [frame, bin, scan point]
    s = w.sensor
    lo = s.bin_t0 + s.bin_width * np.arange(s.n_bins)
    exp = _confocal_plane_bins(D, rw, rh, P, lo, lo + s.bin_width)
    x = per.transpose(1, 0, 2).reshape(s.n_bins, -1)
    mean, se = x.mean(1), x.std(1, ddof=1) / math.sqrt(x.shape[1])
    z = (mean - exp) / se
    assert np.all(np.abs(z) < 4.0), (mean / exp, z)
    assert np.all(np.abs(mean / exp - 1) < 0.06), mean / exp


def test_confocal_plane_restir_matches_closed_form(oracle_lib):
    """ToF ReSTIR with temporal and spatial reuse on the confocal scan: the
    shifted paths end at the destination's own laser spot (the light vertex
    moves with the scan point), and the mean over seeds is the closed form.
    The first bin holds the paths whose length is stationary at the foot
    point of the scan point; without the round-trip check of the shift,
    Newton iterations that fail or land on another root in one direction only
    bias it upward (about +18%, z about 6 here)."""
    D, rw, rh, P = 1.0, 0.8, 0.5, 2.0
    vals = []
    for seed in range(16):
        w = scenes.nlos_plane(depth=D, wall_albedo=rw, albedo=rh, intensity=P, scan=24, frames=3, seed=seed)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        for fr in w.frames:
            out = o.render(fr)["hist"]
        st = o.stats()
        o.close()
        vals.append(out.reshape(w.sensor.n_bins, -1))
    assert st["newton_converged"] > 0.5 * st["newton_attempts"] > 0
    s = w.sensor
    x = np.concatenate(vals, axis=1)                                      # [bin, seed x scan point]
    # scan points of one seed are correlated through reuse: seeds are the samples
    per_seed = np.array([v.mean(1) for v in vals])                        # [seed, bin]
    lo = s.bin_t0 + s.bin_width * np.arange(s.n_bins)
    exp = _confocal_plane_bins(D, rw, rh, P, lo, lo + s.bin_width)
    mean = x.mean(1)
    se = per_seed.std(0, ddof=1) / math.sqrt(per_seed.shape[0])
    z = (mean - exp) / se
    assert np.all(np.abs(z) < 4.0), (mean / exp, z)
    assert np.all(np.abs(mean / exp - 1) < 0.1), mean / exp
