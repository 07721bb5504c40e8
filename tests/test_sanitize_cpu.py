"""Host code under AddressSanitizer, LeakSanitizer and UBSan, on the CPU.

* The oracle: oracle/ghn_oracle.cpp with tests/cpu/oracle_sanitize.cpp, built with g++
  -fsanitize=address,undefined, runs every exported function on seeded inputs.
* The library's host layer: paper_2004_02290_amd/sanitize/host_sanitize (built by
  __graft_entry__.build(): the host-only sources compiled with the sanitizers, linked
  with the ordinary kernels) runs every entry point's argument checks; with a GPU it
  also runs every entry point and the GHN_FAULT failure paths (tests/test_gpu_sanitize.py).
Any report aborts the run with a non-zero status."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUPP = os.path.join(ROOT, "tests", "cpu", "lsan_hip.supp")


def sanitizer_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = "suppressions=" + SUPP
    env.pop("GHN_FAULT", None)
    return env


def host_sanitize_exe():
    from paper_2004_02290_amd import _build
    if not os.path.exists(_build.SAN_EXE):
        _build.build_sanitized()
    return _build.SAN_EXE


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fopenmp",
                           os.path.join(ROOT, "oracle", "ghn_oracle.cpp"),
                           os.path.join(ROOT, "tests", "cpu", "oracle_sanitize.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, env=sanitizer_env(), timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "oracle sanitize ok" in r.stdout


def test_host_layer_under_sanitizers():
    r = subprocess.run([host_sanitize_exe()], capture_output=True, text=True, env=sanitizer_env(), timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "host sanitize ok" in r.stdout
