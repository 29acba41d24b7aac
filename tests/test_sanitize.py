"""The oracle and the C-ABI host layer under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU).  The oracle: gcc builds oracle/los_oracle.c with the driver
tests/sanitize_oracle_driver.c (every entry point on small grids, edge and rejected
arguments).  The host layer: see test_capi_host_under_asan_ubsan.  Each run must finish with
no sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fno-fast-math",
           "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "los_oracle.c"),
           os.path.join(ROOT, "tests", "sanitize_oracle_driver.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("no sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ERROR: AddressSanitizer" not in run.stderr
    assert "runtime error" not in run.stderr


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_capi_host_under_asan_ubsan(tmp_path):
    """The C-ABI host layer (los_api.cpp, batch_api.cpp, emu_api.cpp) built with
    AddressSanitizer and UndefinedBehaviorSanitizer on its host side (the device code of
    every source, and the other translation units, as the library builds them), linked with
    tests/sanitize_capi_driver.cpp: every entry point with NULL handles, NULL arrays and bad
    sizes, and emu_load on refused files; runs without a GPU, with no sanitizer report."""
    build_dir = os.path.join(ROOT, "_build")
    others = [os.path.join(build_dir, f) for f in sorted(os.listdir(build_dir))
              if f.endswith(".o") and f not in ("los_api.cpp.o", "batch_api.cpp.o",
                                                 "emu_api.cpp.o")] if os.path.isdir(build_dir) else []
    if not others:
        pytest.skip("the library objects are not built (paper_2509_25110_amd.build)")
    hipcc = "/opt/rocm/bin/hipcc"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", *san, "-Xarch_host",
             "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
             "-I" + os.path.join(ROOT, "include"),
             "-I" + os.path.join(ROOT, "paper_2509_25110_amd", "csrc")]
    srcs = [os.path.join(ROOT, "paper_2509_25110_amd", "csrc", f)
            for f in ("los_api.cpp", "batch_api.cpp", "emu_api.cpp")]
    srcs.append(os.path.join(ROOT, "tests", "sanitize_capi_driver.cpp"))
    objs = []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([hipcc, *flags, "-x", "hip", "-c", src, "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        objs.append(obj)
    exe = str(tmp_path / "capi_sanitized")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", *san, *objs, *others, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env,
                         timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ERROR: AddressSanitizer" not in run.stderr
    assert "runtime error" not in run.stderr
