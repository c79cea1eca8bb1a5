"""Qualitative behaviour the paper reports, checked on the oracle.

Sec. 6, effect of time-gate width: the reuse success rate of naive
(length-unaware) reuse collapses for narrow gates and grows with the gate
width, while the path-length-aware shift stays roughly constant, and for very
wide gates is slightly below naive reuse (Newton failures and new occlusion).

Sec. 6, Table tab:newton_statistics (stored in tests/golden): the Newton
statistics fall within the band the paper prints across its scenes.
"""
import os

import pytest

from paper_2605_11536_amd import scenes


def _success_rate(oracle_lib, gate_width, mode):
    w = scenes.cornell_box(width=48, height=48, frames=3, gate_width=gate_width, shift_mode=mode,
                           spatial_radius=4)
    o = oracle_lib.Oracle(w.scene, w.sensor)
    for fr in w.frames:
        o.render(fr)
    s = o.stats()
    o.close()
    return s["shifts_ok"] / max(1, s["shifts"])


def test_gate_width_success_rate_trend(oracle_lib):
    widths = [0.02, 0.05, 0.2, 0.5, 1.0]
    naive = [_success_rate(oracle_lib, g, scenes.SHIFT_NAIVE) for g in widths]
    ours = [_success_rate(oracle_lib, g, scenes.SHIFT_PATHLEN) for g in widths]
    print("naive", naive, "pathlen", ours)
    # naive reuse: monotone in the gate width, collapsing at narrow gates
    assert all(b >= a - 0.02 for a, b in zip(naive, naive[1:]))
    assert naive[-1] > 2.5 * naive[0]
    # path-length-aware shift: roughly flat, far better at narrow gates
    assert max(ours) - min(ours) < 0.15
    assert ours[0] > 2.0 * naive[0]
    # and not better than naive at the widest gate
    assert ours[-1] <= naive[-1] + 0.02


def _paper_table():
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "newton_statistics.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, it, sr, asr = line.split()
                rows.append((name, float(it), float(sr), float(asr)))
    return rows


def test_newton_statistics_in_the_papers_band(oracle_lib):
    """Plausibility band of the Newton statistics (Sec. 6, Table
    tab:newton_statistics; the paper's scenes are not available, so this is
    a band, not parity): on the box with a spatial neighbour radius of 2 px
    at 64^2 (about the paper's 30 px relative to its image size) the mean
    iterations per converged solve, the Newton success rate and the actual
    success rate fall within the range the paper prints across its scenes,
    and the actual rate is below the Newton rate as the caption states."""
    rows = _paper_table()
    it_lo, it_hi = min(r[1] for r in rows), max(r[1] for r in rows)
    sr_lo, asr_lo = min(r[2] for r in rows), min(r[3] for r in rows)
    tot = {}
    for seed in range(2):
        w = scenes.cornell_box(width=64, height=64, frames=4, seed=seed, gate_center=4.0, gate_width=0.1,
                               spatial_radius=2)
        o = oracle_lib.Oracle(w.scene, w.sensor)
        for fr in w.frames:
            o.render(fr)
        for k, v in o.stats().items():
            tot[k] = tot.get(k, 0) + v
        o.close()
    iters = tot["newton_iters"] / tot["newton_converged"]
    sr = tot["newton_converged"] / tot["newton_attempts"]
    asr = tot["newton_paths_ok"] / tot["newton_attempts"]
    assert tot["newton_attempts"] > 1000
    assert it_lo - 0.2 <= iters <= it_hi + 0.2, iters
    assert sr >= sr_lo - 0.05, sr
    assert asr_lo - 0.05 <= asr < sr, (asr, sr)
