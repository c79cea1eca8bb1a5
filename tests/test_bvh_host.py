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


def test_serving_arena_and_work_plan(tmp_path):
    """The serving arena's best-fit allocator against a brute-force model, and
    the bounds of the reuse passes' work plan (host code, run on the CPU)."""
    csrc = os.path.join(ROOT, "paper_2605_11536_amd", "csrc")
    exe = tmp_path / "host_logic_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", csrc, os.path.join(ROOT, "tests", "cpp", "host_logic_check.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout[-2000:]
