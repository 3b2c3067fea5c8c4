"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (C, gcc) and the library's host code (setup.cpp with gcc; api.hip
and kernels.hip compiled for the host side only as relocatable device code,
the sanitizers on the host pass) are built into a temporary directory with the drivers in
tests/host_sanitize/ and run on valid and invalid parameters: 2-D and 3-D,
odd counts, one-sided layers, the polynomial smoother, Galerkin operators,
the complex shift, every oracle entry point.  Any memory error or undefined
operation fails the run.  The HIP runtime's own allocations are not leak
checked (it keeps state until exit); the oracle's are."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_1012_5379_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "ora_san"
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "oracle"),
          os.path.join(ROOT, "oracle", "csg_oracle.c"), os.path.join(HERE, "ora_driver.c"), "-lm", "-o", str(exe)])
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([str(exe)], env=env)
    assert "oracle driver: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None, reason="hipcc or g++ not available")
def test_library_host_code_under_sanitizers(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    host_san = [f for flag in SAN for f in ("-Xarch_host", flag)]
    quiet = ["-Wno-unused-value", "-Wno-unused-result"]
    objs = []
    for src in ("api.hip", "kernels.hip"):
        # host side only, as relocatable device code so the link needs no device image
        o = str(tmp_path / (src + ".o"))
        _run([HIPCC, "-std=c++17", "-O1", "-g", "-fPIC", "--offload-arch=gfx950", "-fgpu-rdc", "--offload-host-only",
              *host_san, *quiet, *inc, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src, out in (("setup.cpp", "setup.o"), (os.path.join(HERE, "lib_driver.cpp"), "driver.o")):
        o = str(tmp_path / out)
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        _run(["g++", "-std=c++17", "-O1", "-g", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *inc,
              "-c", path, "-o", o])
        objs.append(o)
    exe = str(tmp_path / "lib_san")
    _run([HIPCC, "--offload-arch=gfx950", "-fgpu-rdc", "--hip-link", *host_san, *objs, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([exe], env=env)
    assert "library host driver: ok" in r.stdout
