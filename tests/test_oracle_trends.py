"""Qualitative behaviour the paper reports, checked on the oracle.

Sec. 6, effect of time-gate width: the reuse success rate of naive
(length-unaware) reuse collapses for narrow gates and grows with the gate
width, while the path-length-aware shift stays roughly constant, and for very
wide gates is slightly below naive reuse (Newton failures and new occlusion).
"""
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
