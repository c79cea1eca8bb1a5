"""The host builder of the 4-wide tree topology (no GPU needed: host code
compiled with hipcc and run on the CPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bvh_host_builder_structure(tmp_path):
    csrc = os.path.join(ROOT, "paper_2605_11536_amd", "csrc")
    exe = tmp_path / "bvh_host_check"
    subprocess.run(["hipcc", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(ROOT, "tests", "cpp", "bvh_host_check.cpp"), "-x", "hip",
                    os.path.join(csrc, "bvh_host.hip"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert out.strip() == "ok", out
