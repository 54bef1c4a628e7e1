"""Host logic of the serving loop: the FIFO device-arena ring (csrc/ib_ring.h), built with
g++ and run on the CPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ring_allocator(tmp_path):
    exe = tmp_path / "ring_test"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2012_06646_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "ring_test.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"
