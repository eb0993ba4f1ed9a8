"""Sanitizer builds, CPU only.  The oracle with AddressSanitizer and
UndefinedBehaviorSanitizer: a C driver calls every entry point on small seeded
inputs, including the threaded bucketed search, and checks it against the flat
search.  The library's host code (built without its device code) with
AddressSanitizer + UndefinedBehaviorSanitizer and with ThreadSanitizer: a
driver runs the request server in its fake mode from several threads, the
load balancing and the workspace footprint."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "asan_oracle")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", exe, os.path.join(HERE, "asan_oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "asci_oracle.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="3")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(p.stdout)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["prims.hip", "search.hip", "bucket.hip", "energy.hip", "eigen.hip", "loop.hip", "server.hip", "graph.hip",
           "tune.hip", "noalloc.hip", "api.hip"]


def _host_build(tmp_path, san):
    """The library and the driver, one executable, each sanitizer flag given
    to the host compiler only (the device code is built as usual, never run)."""
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Xarch_host", "-fno-omit-frame-pointer"]
    for f in san:
        flags += ["-Xarch_host", f]
    csrc = os.path.join(ROOT, "paper_2303_05688_amd", "csrc")
    objs = []

    def one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], check=True,
                       capture_output=True)
        return obj

    srcs = [os.path.join(csrc, x) for x in SOURCES] + [os.path.join(HERE, "host_sanitizer_driver.cpp")]
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(one, srcs))
    exe = str(tmp_path / "host_driver")
    subprocess.run([HIPCC, *flags, "-o", exe, *objs, "-lpthread"], check=True,
                   capture_output=True)
    return exe


def _run(exe, env):
    p = subprocess.run([exe], capture_output=True, text=True, env=dict(os.environ, **env), timeout=600)
    print(p.stdout)
    assert p.returncode == 0, p.stdout + p.stderr
    return p


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    exe = _host_build(tmp_path, ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"])
    p = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_thread_sanitizer(tmp_path):
    exe = _host_build(tmp_path, ["-fsanitize=thread"])
    p = _run(exe, {"TSAN_OPTIONS": "halt_on_error=1"})
    assert "WARNING: ThreadSanitizer" not in p.stderr, p.stderr
