"""AddressSanitizer + UndefinedBehaviorSanitizer build of the library's host
code, driven by tests/host/sanitize_driver.cpp through the C ABI.

Every ``csrc/*.cpp`` file (the host-side algorithms and the C ABI) is
recompiled with host-only sanitizer instrumentation (device code is built
without it); the ``.hip`` objects of the regular build are linked as they are.
The driver runs what needs no GPU: the two- and one-site segment schedules
over random partitions, the sum-of-exponentials fit over exponents, term
counts and ranges (with and without refinement), and the argument checks.
A sanitizer report or a failed invariant fails the test.  CPU only.
"""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1912_06127_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
OUT = os.path.join(BUILD, "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
RT_DIRS = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux"))
HOST_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan",
            *("-Wl,-rpath," + d for d in RT_DIRS)]
LIBS = ["-L/opt/rocm/lib", "-lamdhip64", "-lrocsolver", "-lrocblas", "-lrocprofiler-sdk-roctx",
        "-Wl,-rpath,/opt/rocm/lib"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def _hip_objects():
    objs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src):
            from paper_1912_06127_amd.build import build
            build(verbose=False)
        objs.append(obj)
    return objs


@pytest.fixture(scope="module")
def driver():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not installed")
    os.makedirs(OUT, exist_ok=True)
    objs = _hip_objects()
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < max(
                os.path.getmtime(src), *(os.path.getmtime(h) for h in glob.glob(os.path.join(CSRC, "*.hpp")))):
            _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-I" + os.path.join(ROOT, "include"), *SAN, "-x", "hip", "-c", src, "-o", obj])
        objs.append(obj)
    lib = os.path.join(OUT, "libtdvp_sanitize.so")
    _run([CLANG, "-shared", "-o", lib, *objs, *HOST_SAN, *LIBS])
    exe = os.path.join(OUT, "sanitize_driver")
    _run([CLANG, "-O1", "-g", "-std=c++17", *HOST_SAN, "-I" + os.path.join(ROOT, "include"),
          os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp"), "-o", exe, lib, *LIBS,
          "-Wl,-rpath," + OUT])
    return exe


def test_host_logic_is_clean_under_asan_and_ubsan(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-6000:]
    assert "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert "0 failed checks" in r.stdout
