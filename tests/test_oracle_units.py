"""Pins of the CPU oracle's building blocks against things other than itself.

* Philox4x64-10 against numpy's independent implementation (library routine).
* BVH closest hit against brute force over every primitive.
* Surface charts against the lattice vertices and analytic sphere formulas.
* The Newton shift (Sec. 4.3) against the confocal radial closed form, finite
  differences of the composite map xi -> xi', the gate constraint, the
  identity shift and the round trip (bijectivity).
* Weighted reservoir sampling (Sec. 3.2.4) selection frequencies (chi-square).
"""
import math

import numpy as np
import pytest

from paper_2605_11536_amd import scenes


# --------------------------------------------------------------------------
# Philox
# --------------------------------------------------------------------------

def test_philox_matches_numpy_bit_exact(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] = ctr[0] * 2 + 1   # exercise the top bit through the carry below
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        # numpy's Philox increments the counter before producing a block
        prev = list(ctr)
        prev[0] = (prev[0] - 1) % 2**64
        bg = np.random.Philox(key=key)
        st = bg.state
        st["state"]["counter"] = np.array(prev, dtype=np.uint64)   # exact (a list goes through float64)
        st["buffer_pos"] = 4
        bg.state = st
        ref = bg.random_raw(4)
        got = oracle_lib.philox4x64(ctr, key)
        assert np.array_equal(ref.astype(np.uint64), got), (ctr, key)


def test_philox_uniforms_are_uniform(oracle_lib):
    n = 20000
    us = np.empty(n)
    for i in range(n // 4):
        x = oracle_lib.philox4x64([i, 3, 1 << 56, 0], [0, 0])
        us[4 * i: 4 * i + 4] = (x >> np.uint64(40)).astype(np.float64) / 2.0**24
    assert us.min() >= 0.0 and us.max() < 1.0
    hist, _ = np.histogram(us, bins=20, range=(0, 1))
    chi2 = ((hist - n / 20) ** 2 / (n / 20)).sum()
    assert chi2 < 43.8      # 99.9% quantile of chi2(19)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def _rand_rays(rng, n, lo, hi):
    o = rng.uniform(lo, hi, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


@pytest.mark.parametrize("which", ["glossy", "nlos", "box"])
def test_bvh_matches_brute_force(oracle_lib, which):
    if which == "glossy":
        w = scenes.glossy_dynamic(width=8, height=8, frames=2, ground_cells=40, sphere_nu=16, sphere_nv=10)
        lo, hi = [-5, -0.5, -5], [5, 2, 5]
    elif which == "nlos":
        w = scenes.nlos_confocal(scan=8, frames=2, torus_nu=60, torus_nv=24)
        lo, hi = [-1, -1, 0.05], [1, 1, 1.5]
    else:
        w = scenes.cornell_box(width=8, height=8)
        lo, hi = [-0.95] * 3, [0.95] * 3
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    o.load_frame(w.frames[-1])
    rng = np.random.default_rng(1)
    org, dirs = _rand_rays(rng, 1500, lo, hi)
    hits = 0
    for a, d in zip(org, dirs):
        p1, r1 = o.trace(a, d, brute=False)
        p2, r2 = o.trace(a, d, brute=True)
        assert p1 == p2
        if p1 >= 0:
            hits += 1
            assert r1[0] == pytest.approx(r2[0], rel=1e-12)
            # the chart point of the hit reproduces the ray point
            on, p, _, _, _ = o.chart(int(r1[1]), r1[2:4])
            assert np.allclose(p, a + r1[0] * d, atol=1e-9)
    assert hits > 200
    o.close()


def test_grid_chart_reproduces_lattice_and_sphere_formula(oracle_lib):
    w = scenes.glossy_dynamic(width=8, height=8, frames=3, ground_cells=20, sphere_nu=12, sphere_nv=8)
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    fr = w.frames[2]
    o.load_frame(fr)
    sc = w.scene
    rng = np.random.default_rng(3)
    for obj in range(sc.num_objects):
        nu, nv, wu, wv, off = sc.obj_grid[obj]
        m = fr.xforms[obj].astype(np.float64).reshape(3, 4)
        for _ in range(10):
            i, j = rng.integers(0, nu + 1), rng.integers(0, nv + 1)
            loc = sc.vertices[off + j * (nu + 1) + i].astype(np.float64)
            on, p, ju, jv, n = o.chart(obj, [float(i), float(j)])
            assert np.allclose(p, m[:, :3] @ loc + m[:, 3], atol=1e-12)
            if on:   # polar rows of a latitude/longitude lattice are degenerate
                assert abs(np.linalg.norm(n) - 1) < 1e-12
    # analytic sphere chart of the box scene
    w = scenes.cornell_box(width=8, height=8)
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    o.load_frame(w.frames[0])
    m = w.frames[0].xforms[5].astype(np.float64).reshape(3, 4)
    for th, ph in [(0.3, 0.2), (1.5, 4.0), (2.9, 6.0)]:
        on, p, ju, jv, n = o.chart(5, [th, ph])
        loc = 0.3 * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        assert on
        assert np.allclose(p, m[:, :3] @ loc + m[:, 3], atol=1e-12)
        h = 1e-6
        _, pp, _, _, _ = o.chart(5, [th + h, ph])
        _, pm, _, _, _ = o.chart(5, [th - h, ph])
        assert np.allclose((pp - pm) / (2 * h), ju, atol=1e-8)


# --------------------------------------------------------------------------
# Newton shift (Sec. 4.3)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def wall(oracle_lib):
    """The NLOS relay wall: a 2x2 planar 1x1-cell grid at z=0 (chart in cell
    units: one cell = 2 scene units)."""
    w = scenes.nlos_confocal(scan=8, frames=1, torus_nu=20, torus_nv=8)
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    o.load_frame(w.frames[0])
    yield o
    o.close()


@pytest.fixture(scope="module")
def box(oracle_lib):
    w = scenes.cornell_box(width=8, height=8)
    o = oracle_lib.Oracle(w.scene, w.sensor, num_threads=1)
    o.load_frame(w.frames[0])
    yield o
    o.close()


def _pos(o, obj, xi):
    return o.chart(obj, xi)[1]


def test_confocal_radial_closed_form(wall):
    """p1 = p2 = g above a plane: the average-gradient gauge moves p radially
    from the foot point of g and |det dxi'/dxi| = r'/r exactly."""
    g = np.array([0.1, -0.2, 0.7])
    for xi, dl in [((0.65, 0.6), 0.15), ((0.3, 0.75), -0.1), ((0.8, 0.2), 0.05)]:
        p = _pos(wall, 0, xi)
        r = np.linalg.norm(g - p)
        out = wall.newton(0, xi, g, g, 0.0, g, g, 0.0, dl, tol=1e-13, max_iter=20)
        assert out["ok"]
        pn = _pos(wall, 0, out["xi"])
        rn = np.linalg.norm(g - pn)
        assert rn == pytest.approx(r + dl / 2, abs=1e-12)
        foot = np.array([g[0], g[1], 0.0])
        a, b = p - foot, pn - foot
        assert abs(a[0] * b[1] - a[1] * b[0]) < 1e-10 * np.linalg.norm(a) * np.linalg.norm(b)
        assert np.dot(a, b) > 0
        assert out["det_dxi"] == pytest.approx((r + dl / 2) / r, rel=1e-10)
        assert out["det_area"] == pytest.approx((r + dl / 2) / r, rel=1e-10)


def _fd_det(o, obj, xi, a_s, b_s, c_s, a_d, b_d, c_d, dl, h):
    cols = []
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        plus = o.newton(obj, np.array(xi) + e, a_s, b_s, c_s, a_d, b_d, c_d, dl, tol=1e-14, max_iter=30)
        minus = o.newton(obj, np.array(xi) - e, a_s, b_s, c_s, a_d, b_d, c_d, dl, tol=1e-14, max_iter=30)
        assert plus["ok"] and minus["ok"]
        cols.append((plus["xi"] - minus["xi"]) / (2 * h))
    return abs(np.linalg.det(np.array(cols).T))


@pytest.mark.parametrize("case", range(4))
def test_newton_jacobian_matches_finite_differences(box, case):
    """|det dxi'/dxi| from implicit differentiation equals the central
    difference of the composite map (planar chart and the curved sphere chart,
    which exercises the curvature term Q)."""
    rng = np.random.default_rng(100 + case)
    if case < 2:
        obj, xi = 0, (0.3 + 0.4 * rng.random(), 0.3 + 0.4 * rng.random())   # back wall
        a_s = np.array([0.3, -0.8, 0.2]) + 0.1 * rng.normal(size=3)
        b_s = np.array([0.0, 0.0, 1.0])
        a_d = a_s + np.array([0.08, 0.05, -0.03])
        b_d = b_s + (0.0 if case == 0 else np.array([0.05, 0.0, 0.0]))
        h = 1e-6
    else:
        obj, xi = 5, (1.2 + 0.3 * rng.random(), 0.5 + 0.5 * rng.random())   # sphere
        p = _pos(box, obj, xi)
        _, _, _, _, n = box.chart(obj, xi)
        a_s = p + 0.8 * n + np.array([0.1, 0.2, 0.0])
        b_s = p + 0.9 * n + np.array([-0.2, 0.05, 0.1])
        a_d = a_s + np.array([0.03, -0.02, 0.02])
        b_d = b_s
        h = 1e-6
    c_s, c_d = 0.7, (0.75 if case < 2 else 0.71)
    dl = 0.02 * (case % 2) if case < 2 else 0.004 * (case % 2)
    out = box.newton(obj, xi, a_s, b_s, c_s, a_d, b_d, c_d, dl, tol=1e-14, max_iter=30)
    assert out["ok"], out
    fd = _fd_det(box, obj, xi, a_s, b_s, c_s, a_d, b_d, c_d, dl, h)
    assert out["det_dxi"] == pytest.approx(fd, rel=1e-5)
    # surface-area Jacobian |det dp'/dp| from 3-D positions only: the area of
    # the image of a small chart patch divided by the area of the patch
    d_src, d_dst = [], []
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        xp = box.newton(obj, np.array(xi) + e, a_s, b_s, c_s, a_d, b_d, c_d, dl, tol=1e-14, max_iter=30)["xi"]
        xm = box.newton(obj, np.array(xi) - e, a_s, b_s, c_s, a_d, b_d, c_d, dl, tol=1e-14, max_iter=30)["xi"]
        d_dst.append(_pos(box, obj, xp) - _pos(box, obj, xm))
        d_src.append(_pos(box, obj, np.array(xi) + e) - _pos(box, obj, np.array(xi) - e))
    ratio = np.linalg.norm(np.cross(*d_dst)) / np.linalg.norm(np.cross(*d_src))
    assert out["det_area"] == pytest.approx(ratio, rel=1e-5)


def test_newton_gate_constraint_and_identity(box):
    """Converged shifts satisfy |l(y') - l(x) - dl| <= 1e-6 l (recomputed from
    chart positions); the identity shift takes 0 iterations with J = 1."""
    rng = np.random.default_rng(7)
    nconv = 0
    for trial in range(60):
        obj = int(rng.integers(0, 5))
        xi = (0.2 + 0.6 * rng.random(), 0.2 + 0.6 * rng.random())
        p = _pos(box, obj, xi)
        _, _, _, _, n = box.chart(obj, xi)
        a_s = p + rng.uniform(0.6, 1.2) * n + 0.3 * rng.normal(size=3)
        b_s = np.array([0.0, 0.0, 1.0])
        a_d = a_s + 0.05 * rng.normal(size=3)
        c_s, c_d = 1.0, 1.0 + 0.02 * rng.normal()
        dl = 0.05 * rng.normal()
        L = c_s + np.linalg.norm(a_s - p) + np.linalg.norm(b_s - p)
        out = box.newton(obj, xi, a_s, b_s, c_s, a_d, b_d := b_s, c_d, dl, tol=1e-6 * L, max_iter=8)
        if out["ok"]:
            nconv += 1
            q = _pos(box, obj, out["xi"])
            Ln = c_d + np.linalg.norm(a_d - q) + np.linalg.norm(b_d - q)
            assert abs(Ln - L - dl) <= 1e-6 * L
        ident = box.newton(obj, xi, a_s, b_s, c_s, a_s, b_s, c_s, 0.0, tol=1e-9, max_iter=5)
        assert ident["ok"] and ident["iters"] == 0
        assert np.array_equal(ident["xi"], np.array(xi))
        assert ident["det_dxi"] == pytest.approx(1.0, abs=1e-14)
    assert nconv >= 40


def test_newton_round_trip_is_bijective(box):
    """T_{q->j}(T_{j->q}(x)) = x within tolerance and J_fwd * J_inv = 1."""
    rng = np.random.default_rng(11)
    checked = 0
    for trial in range(60):
        obj = int(rng.integers(0, 6))
        if obj == 5:
            xi = (1.0 + 1.0 * rng.random(), 6.0 * rng.random())
        else:
            xi = (0.2 + 0.6 * rng.random(), 0.2 + 0.6 * rng.random())
        p = _pos(box, obj, xi)
        _, _, _, _, n = box.chart(obj, xi)
        a_s = p + 0.9 * n + 0.2 * rng.normal(size=3)
        b_s = p + 0.7 * n + 0.2 * rng.normal(size=3)
        a_d = a_s + 0.04 * rng.normal(size=3)
        b_d = b_s + 0.02 * rng.normal(size=3)
        c_s, c_d, dl = 0.5, 0.52, 0.01 * rng.normal()
        fwd = box.newton(obj, xi, a_s, b_s, c_s, a_d, b_d, c_d, dl, tol=1e-13, max_iter=20)
        if not fwd["ok"]:
            continue
        inv = box.newton(obj, fwd["xi"], a_d, b_d, c_d, a_s, b_s, c_s, -dl, tol=1e-13, max_iter=20)
        assert inv["ok"]
        assert np.allclose(inv["xi"], xi, atol=1e-9)
        assert fwd["det_dxi"] * inv["det_dxi"] == pytest.approx(1.0, rel=1e-6)
        checked += 1
    assert checked >= 25


def test_printed_sign_of_hessian_term_would_fail(box):
    """Guard for the reading of dF2/dxi': the finite-difference Jacobian of
    the confocal case equals r'/r; a Hessian term of the opposite sign would
    give a different determinant (checked here on the closed form only)."""
    g = np.array([0.0, 0.0, 1.0])
    xi = (0.65, 0.6)        # back wall chart, cell units of 2
    p = _pos(box, 0, xi)
    # the back wall is z=-1; move g to make p1 = p2 = g in front of it
    out = box.newton(0, xi, g, g, 0.0, g, g, 0.0, 0.15, tol=1e-13, max_iter=20)
    assert out["ok"]
    r = np.linalg.norm(g - p)
    assert out["det_dxi"] == pytest.approx((r + 0.075) / r, rel=1e-10)


# --------------------------------------------------------------------------
# weighted reservoir sampling (Sec. 3.2.4)
# --------------------------------------------------------------------------

def test_wrs_selection_frequencies(oracle_lib):
    w = np.array([0.5, 3.0, 0.0, 1.5, 2.0, 0.25])
    rng = np.random.default_rng(2)
    n = 40000
    counts = np.zeros(len(w))
    for _ in range(n):
        u = rng.random(len(w))
        sel, ws = oracle_lib.wrs(w, u)
        assert ws == pytest.approx(w.sum())
        counts[sel] += 1
    exp = n * w / w.sum()
    mask = exp > 0
    assert counts[~mask].sum() == 0
    chi2 = ((counts[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    assert chi2 < 20.5      # 99.9% quantile of chi2(4)


def test_mis_weights_partition_of_unity(oracle_lib):
    """P7: at any path, the MIS weights of all techniques of a spatial reuse
    sum to one (Sec. 3.2.3: the condition for GRIS to be unbiased), for the
    generalized balance heuristic and for pairwise MIS, with unequal
    confidences, neighbours without a pixel and failed shifts; plus weights
    worked by hand."""
    mw = oracle_lib.mis_weights
    rng = np.random.default_rng(2)
    for mode in (0, 1):
        for _ in range(300):
            K = int(rng.integers(1, 9))
            M = rng.uniform(0.5, 20.0, K)
            M[rng.random(K) < 0.2] = -1.0
            d = rng.exponential(1.0, K) * (rng.random(K) > 0.25)
            w = mw(mode, M, float(rng.uniform(0.5, 20.0)), d, float(rng.exponential(1.0) + 1e-3))
            assert abs(w.sum() - 1.0) < 1e-12, (mode, w)
            assert np.all(w >= 0.0) and np.all(w[1:][M < 0] == 0.0)
    M, mq, d, dc = [1.0, 3.0], 2.0, [0.5, 0.25], 1.0
    # balance heuristic: M_t d_t / (mq dc + sum M_l d_l), den = 3.25
    assert np.allclose(mw(0, M, mq, d, dc), [2 / 3.25, 0.5 / 3.25, 0.75 / 3.25], rtol=1e-14)
    # pairwise: mq split in two parts of 1; pair weights (M_l + 1) / 6
    assert np.allclose(mw(1, M, mq, d, dc), [38 / 63, 1 / 9, 2 / 7], rtol=1e-14)
    # one neighbour: pairwise is the balance heuristic
    assert np.allclose(mw(1, [3.0, -1.0], 2.0, [0.4, 0.0], 0.7), mw(0, [3.0, -1.0], 2.0, [0.4, 0.0], 0.7))


def test_merge_diagnostics_are_consistent(oracle_lib):
    """The merge diagnostics (a report of the resampling weights, not part of
    the estimate): per merge the effective sample count lies between 1 and
    the number of candidates with a positive weight, which is at most the
    number present, at most k + 1; the canonical share is a fraction.  Three
    frames of the box with temporal and spatial reuse."""
    from oracle.oracle import Oracle
    w = scenes.cornell_box(frames=3)
    o = Oracle(w.scene, w.sensor)
    for fr in w.frames:
        o.render(fr)
    d = o.merge_diag()
    o.close()
    for name, kmax in (("temporal", 2), ("spatial", w.sensor.spatial_k + 1)):
        r = d[name]
        n = r["merges"]
        assert n > 0, name
        assert n - 1e-9 <= r["ess"] <= r["positive"] + 1e-9, (name, r)
        assert r["positive"] <= r["present"] <= kmax * n, (name, r)
        assert 0.0 <= r["canonical_share"] <= n + 1e-9, (name, r)
    assert d["spatial"]["ess"] > 1.05 * d["spatial"]["merges"]   # spatial reuse does pool candidates
