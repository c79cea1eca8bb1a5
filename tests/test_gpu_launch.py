"""Launch shape of the reuse passes (tof_set_launch_config, tof_autotune):
the results do not depend on it, and tuning leaves no trace but the shape."""
import numpy as np
import pytest

from paper_2605_11536_amd import scenes

pytestmark = pytest.mark.gpu

COUNTS = ("shifts", "shifts_ok", "newton_attempts", "newton_converged", "newton_iters", "newton_paths_ok", "rays",
          "frames", "bvh_overflow", "bad_records")


def _glossy(frames):
    return scenes.glossy_dynamic(width=64, height=64, full_width=512, full_height=512, crop_x0=224, crop_y0=200,
                                 frames=frames)


def test_launch_shape_does_not_change_results():
    """Three frames of the glossy crop with the default shape, with the
    smallest grids (64 shift blocks, 64 visibility blocks), with mixed ones,
    with the visibility kernel compiled for 5 waves per SIMD and merge
    tiles of 1 and 4 tasks, each over many small chunks: outputs
    bit-identical, counters equal."""
    from paper_2605_11536_amd.tof import Renderer
    w = _glossy(3)
    shapes = [(0, 0, 0, 0), (64, 64, 5, 1), (2048, 32768, 5, 4), (4096, 8192, 6, 2)]
    rs = []
    for shape in shapes:
        r = Renderer(w.scene, w.sensor)
        r.set_launch_config(*shape)
        r.set_ray_budget(1)
        rs.append(r)
    assert rs[1].launch_config() == {"shift_blocks": 64, "vis_blocks": 64, "vis_waves": 5, "merge_tasks": 1}
    assert rs[0].launch_config() == {"shift_blocks": 8192, "vis_blocks": 16384, "vis_waves": 6, "merge_tasks": 2}
    for fr in w.frames:
        print(f"case launch shapes frame {fr.index}", flush=True)
        outs = []
        for r in rs:
            r.render(fr)
            outs.append(r.fetch())
        for o in outs[1:]:
            for key in outs[0]:
                assert np.array_equal(outs[0][key], o[key]), (fr.index, key)
    st = [r.stats() for r in rs]
    for s in st[1:]:
        for k in COUNTS:
            assert s[k] == st[0][k], (k, s[k], st[0][k])
    for r in rs:
        r.close()


def test_autotune_leaves_no_trace_but_the_shape():
    """tof_autotune on four frames: it returns one of its candidates, leaves
    the counters as they were, drops the history (the next frame equals a
    fresh context's first frame, bit for bit), and rejects too few frames and
    shapes out of range."""
    from paper_2605_11536_amd.tof import Renderer, TofError
    w = _glossy(5)
    r = Renderer(w.scene, w.sensor)
    r.render(w.frames[0])
    before = r.stats()
    print("case autotune", flush=True)
    cfg = r.autotune(w.frames[:4])
    print("chosen", cfg, flush=True)
    assert cfg["shift_blocks"] in (8192, 4096, 2048) and cfg["vis_blocks"] in (4096, 8192, 16384, 32768)
    assert cfg["vis_waves"] in (5, 6) and cfg["merge_tasks"] in (1, 2, 4)
    assert r.launch_config() == cfg
    after = r.stats()
    for k in COUNTS:
        assert after[k] == before[k], (k, after[k], before[k])
    r.render(w.frames[4])
    got = r.fetch()
    fresh = Renderer(w.scene, w.sensor)
    fresh.render(w.frames[4])
    ref = fresh.fetch()
    for key in ref:
        assert np.array_equal(got[key], ref[key]), key
    with pytest.raises(TofError):
        r.autotune(w.frames[:1])
    for bad in ((100, 0), (16384, 0), (0, 131072), (0, 0, 4, 0), (0, 0, 0, 3)):
        with pytest.raises(TofError):
            r.set_launch_config(*bad)
    assert r.launch_config() == cfg
    r.close()
    fresh.close()
