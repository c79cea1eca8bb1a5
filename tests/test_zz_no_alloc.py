"""tof_render_frame_noalloc: the frame's work space in the library's static
device array gives the same frames as tof_render_frame, bit for bit, on two
calls in a row where the second has the smaller input; a sensor whose work
space cannot fit is refused and the context stays usable."""
import numpy as np
import pytest

from paper_2605_11536_amd import scenes

pytestmark = pytest.mark.gpu


def test_noalloc_matches_render_frame():
    from paper_2605_11536_amd.tof import Renderer
    big = scenes.glossy_dynamic(width=64, height=64, full_width=512, full_height=512, crop_x0=224, crop_y0=200,
                                frames=3)
    small = scenes.cornell_box(width=32, height=32, frames=3, spatial_radius=4)
    ref = {w.name: Renderer(w.scene, w.sensor) for w in (big, small)}
    got = {w.name: Renderer(w.scene, w.sensor) for w in (big, small)}
    for f in range(3):
        for w in (big, small):   # two calls in a row, the second with the smaller frame
            print(f"case noalloc {w.name} frame {f}", flush=True)
            ref[w.name].render(w.frames[f])
            got[w.name].render_noalloc(w.frames[f])
        for w in (big, small):
            a, b = ref[w.name].fetch(), got[w.name].fetch()
            for key in a:
                assert np.array_equal(a[key], b[key]), (w.name, f, key)
            assert np.any(b["hist" if "hist" in b else "image"] != 0)
    for w in (big, small):
        sa, sb = ref[w.name].stats(), got[w.name].stats()
        for k in ("shifts", "shifts_ok", "newton_attempts", "newton_converged", "rays"):
            assert sa[k] == sb[k], (w.name, k)
        ref[w.name].close()
        got[w.name].close()


def test_noalloc_refuses_a_work_space_beyond_the_array():
    from paper_2605_11536_amd.tof import Renderer, TofError
    w = scenes.glossy_dynamic(width=512, height=512, frames=2)   # 67 M pixel-planes: 1 GiB of per-plane parts
    r = Renderer(w.scene, w.sensor)
    with pytest.raises(TofError) as e:
        r.render_noalloc(w.frames[0])
    assert e.value.status == -2
    r.render(w.frames[0])   # the context is untouched
    assert r.stats()["frames"] == 1
    r.close()
