"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU: ``csrc/api.cpp`` (argument validation, hierarchy and footprint
planning, workspace layout) is recompiled with both sanitizers on its host
side only, linked with the in-tree objects of the device code into
``host_sanitizer_driver.cpp``, and run. The driver makes only the calls that
finish on the host (about 36k footprint plans over a sweep of grids, limits,
restarts and batch sizes, every argument check, null handles), so no GPU is
needed; any sanitizer report fails the run."""
import glob
import os
import shlex
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1712_08740_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host side only: the device code is not instrumented
SAN = shlex.split("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                  "-Xarch_host -fno-sanitize-recover=undefined "
                  "-Xarch_host -fno-omit-frame-pointer")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, f"{cmd[0]} failed:\n{r.stderr[-4000:]}"


def test_host_code_is_clean_under_sanitizers(tmp_path):
    if not shutil.which(HIPCC):
        pytest.skip("hipcc not available")
    objs = [o for o in glob.glob(os.path.join(ROOT, "_build", "*.o"))
            if os.path.basename(o) != "api.cpp.o"]
    if not objs:
        pytest.skip("library objects not built (run __graft_entry__.build())")
    inc = [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    api = str(tmp_path / "api.o")
    drv = str(tmp_path / "driver.o")
    exe = str(tmp_path / "driver")
    _run([HIPCC, "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN + inc
         + ["-c", os.path.join(CSRC, "api.cpp"), "-o", api])
    _run([HIPCC, "-O1", "-g", "-std=c++17"] + SAN + inc
         + ["-c", os.path.join(ROOT, "tests", "host_sanitizer_driver.cpp"), "-o", drv])
    _run([HIPCC, "--offload-arch=gfx950"] + SAN + ["-o", exe, drv, api] + sorted(objs))
    env = dict(os.environ,
               # the HIP runtime's own allocations live until exit
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "0 failures" in r.stdout and r.stdout.rstrip().endswith("ok"), out[-4000:]
