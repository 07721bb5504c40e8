"""The end-of-walk guard (a walk that ends without k rows of the index writes the "no
answer" row and raises a fault bit): the header the kernels include, compiled with g++
and run on the CPU.  Nothing here provokes the condition on a GPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_guard_logic_on_cpu(tmp_path):
    exe = str(tmp_path / "guard_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-DGHN_HD=",
                           "-I" + os.path.join(ROOT, "paper_2004_02290_amd", "csrc"),
                           os.path.join(ROOT, "tests", "cpu", "guard_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "guard ok" in r.stdout
