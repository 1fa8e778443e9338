"""The host runtime (csrc/api.cpp with the serving arena of csrc/arena.h) built for the
CPU with AddressSanitizer and UndefinedBehaviorSanitizer (leak checking on) and run
by tests/host/sanitize_driver.cpp: a randomized arena allocate/release sequence and the
host-only C-ABI calls with every heap allocation failing in turn.  No GPU is used;
the kernel launchers are stand-ins (tests/host/launch_stubs.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_07088_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_runtime_under_asan_ubsan(tmp_path):
    out = str(tmp_path)
    common = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
              "-I", CSRC] + SAN
    objs = []
    for src, lang in [(os.path.join(CSRC, "api.cpp"), ["-x", "hip"]),
                      (os.path.join(HOST, "launch_stubs.cpp"), ["-x", "hip"]),
                      (os.path.join(HOST, "sanitize_driver.cpp"), [])]:
        obj = os.path.join(out, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC] + common + lang + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        objs.append(obj)
    exe = os.path.join(out, "sanitize_driver")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950"] + SAN + objs + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    supp = os.path.join(out, "lsan.supp")
    with open(supp, "w") as f:
        # one-time allocations of the HIP and HSA runtimes loaded with the library
        f.write("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:allocator_may_return_null=1",
               LSAN_OPTIONS=f"suppressions={supp}:print_suppressions=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host runtime checks passed" in r.stdout
