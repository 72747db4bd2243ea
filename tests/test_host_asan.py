"""The library's host code under AddressSanitizer (no GPU needed).

The host sources (argument checks, workspace layout, launch set-up, the autotune cache file
parser and writer) are compiled with AddressSanitizer and linked, with the device objects of the
regular build, into a small C program (tests/asan/host_checks.c) that calls every entry point's
rejecting paths and the cache load and save on malformed files. The test passes when the program
reports every expected status and the sanitizer reports no error or leak."""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_17168_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"


def test_host_code_under_address_sanitizer(tmp_path):
    hipcc = _hipcc()
    hip_objs = sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    if len(hip_objs) != len(srcs):        # no regular build yet: make one (device objects)
        from paper_2501_17168_amd import build
        build.build()
        hip_objs = sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
    asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g", "-O1"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    procs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        procs.append(subprocess.Popen([hipcc, *asan, "-std=c++17", *inc, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    drv = str(tmp_path / "host_checks.o")
    procs.append(subprocess.Popen([hipcc, "-x", "c", *asan, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                                   *inc, "-c", os.path.join(ROOT, "tests", "asan", "host_checks.c"), "-o", drv],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, f"{p.args}\n{err[-3000:]}"
    exe = str(tmp_path / "host_checks")
    _run([hipcc, "-Xarch_host", "-fsanitize=address", "-o", exe, drv, *objs, *hip_objs])
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    r = subprocess.run([exe, str(scratch)], capture_output=True, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stderr and "LeakSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host checks passed" in r.stdout
