"""libpsc's host code (psc_host.cpp, psc_server.cpp) under AddressSanitizer
and UndefinedBehaviorSanitizer on the CPU: compiled for the host with the
HIP runtime and the kernel launchers answered by tests/host_stub_hip.cpp
(device buffers become heap blocks, so every copy into or out of them is
bounds-checked, and every launch checks its arguments against the lattice
record), then driven by tests/host_asan_driver.cpp through the C ABI: the
freeze, launch shapes, tape growth, per-launch timing switched on and off as
the benchmark does, read-backs, checkpoint loading, ensembles and the
serving loop.  Any invalid access, undefined behaviour or leak fails it.
The same program under ThreadSanitizer checks the serving loop's two
threads (the builder of admitted jobs and the worker that steps them)
against the submitting thread."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1605_03726_amd", "csrc")


def build_and_run(tmp_path, name, sanitize, env):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / name)
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-pthread", "-Wno-unused-result",
           "-fno-omit-frame-pointer"] + sanitize + [
           "-o", exe,
           os.path.join(CSRC, "psc_host.cpp"), os.path.join(CSRC, "psc_server.cpp"),
           os.path.join(HERE, "host_stub_hip.cpp"), os.path.join(HERE, "host_asan_driver.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, **env))
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "launch check failures 0" in p.stdout
    return p


def test_host_code_is_clean_under_sanitizers(tmp_path):
    build_and_run(tmp_path, "host_asan", ["-fsanitize=address,undefined",
                                          "-fno-sanitize-recover=undefined"],
                  {"ASAN_OPTIONS": "detect_leaks=1"})


def test_host_code_is_free_of_data_races(tmp_path):
    p = build_and_run(tmp_path, "host_tsan", ["-fsanitize=thread"],
                      {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"})
    assert "ThreadSanitizer" not in p.stderr, p.stderr[-4000:]
