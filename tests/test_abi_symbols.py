"""The C ABI library loads and exports every entry point include/tof.h
declares (no GPU needed: nothing here launches device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tof.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tof_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libtof():
    from paper_2605_11536_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return ctypes.CDLL(build.LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("tof_create", "tof_destroy", "tof_scene_upload", "tof_sensor_set", "tof_render_frame",
              "tof_reservoirs_reset", "tof_get_stats", "tof_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(libtof):
    for name in _declared():
        assert hasattr(libtof, name), name


def test_status_strings(libtof):
    libtof.tof_status_string.restype = ctypes.c_char_p
    libtof.tof_status_string.argtypes = [ctypes.c_int]
    assert libtof.tof_status_string(0) == b"ok"
    assert b"budget" in libtof.tof_status_string(-2)
    assert libtof.tof_status_string(-99) == b"unknown status"


def test_binding_struct_layouts_match_header():
    """The ctypes mirrors have one field per C struct member, in order."""
    from paper_2605_11536_amd import tof
    src = open(os.path.join(ROOT, "include", "tof.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    for cname, pycls in (("tof_sensor_desc", tof.tof_sensor_desc), ("tof_frame_desc", tof.tof_frame_desc),
                         ("tof_scene_desc", tof.tof_scene_desc), ("tof_stats", tof.tof_stats)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", src).group(1)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split("*", 1)[1]
            for n in names.split(","):
                n = n.strip().lstrip("*").split("[")[0].strip()
                if n:
                    fields.append(n)
        assert fields == [f[0] for f in pycls._fields_], cname


def test_binding_struct_sizes_and_offsets_match_c(tmp_path):
    """gcc compiles the header; every ctypes mirror has the C size and field
    offsets."""
    import subprocess
    from paper_2605_11536_amd import tof
    structs = {"tof_scene_desc": tof.tof_scene_desc, "tof_sensor_desc": tof.tof_sensor_desc,
               "tof_frame_desc": tof.tof_frame_desc, "tof_stats": tof.tof_stats,
               "tof_history_desc": tof.tof_history_desc, "tof_kernel_work": tof.tof_kernel_work,
               "tof_kernel_times": tof.tof_kernel_times, "tof_bvh_info": tof.tof_bvh_info,
               "tof_launch_config": tof.tof_launch_config}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tof.h"', "int main(void) {"]
    for cname, pycls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in pycls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, pycls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(pycls), cname
        for fname, _ in pycls._fields_:
            assert got[(cname, fname)] == getattr(pycls, fname).offset, (cname, fname)
