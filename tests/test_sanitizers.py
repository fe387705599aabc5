"""AddressSanitizer and UndefinedBehaviorSanitizer builds of host code (no GPU).

* The C oracle: every entry point on small lattices of each geometry, equation of state and
  adhesion form (tests/sanitize/oracle_driver.c), leak detection on.
* The host side of liblbm: parameter validation, workspace layouts, the Carnahan-Starling and
  Eq. (15) solvers, rejected buffers and handles (tests/sanitize/host_api_driver.cpp). The C-ABI
  layer is compiled with the sanitizers on its host pass only (its device code builds as usual)
  and linked with the kernel objects of the regular build, whose launchers the driver never
  reaches.
(The device code's index maps run under the same sanitizers in tests/test_emu_index_maps.py.)
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
PKG = os.path.join(ROOT, "paper_1410_2569_amd")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "passed: 0 failure(s)" in r.stdout


@pytest.mark.skipif(not (shutil.which(HIPCC) and shutil.which(CLANGXX)), reason="no ROCm compilers")
def test_library_host_code_under_sanitizers(tmp_path):
    objs = [os.path.join(PKG, "_build", f"{s}.o") for s in ("lbm_kernels", "lbm_adjoint",
                                                             "lbm_batch")]
    if not all(os.path.exists(o) for o in objs):
        from paper_1410_2569_amd import build
        build.build()
    api = str(tmp_path / "lbm_api_san.o")
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC",
                           "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
                           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-c",
                           os.path.join(PKG, "csrc", "lbm_api.hip"), "-o", api])
    drv = str(tmp_path / "driver.o")
    subprocess.check_call([CLANGXX, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-c",
                           os.path.join(SAN, "host_api_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "host_api_driver")
    subprocess.check_call([CLANGXX, "-fsanitize=address,undefined", drv, *objs, api,
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "passed: 0 failure(s)" in r.stdout
