"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The FP64 oracle (plain C) is built with gcc and both sanitizers and driven
  through every entry point on small inputs (tests/sanitize/oracle_driver.c),
  leak detection on.
- The library's host code (argument and CSR checks, greedy initialisation,
  footprint model, error messages) is built with the sanitizers on the host
  side only (device code is compiled normally and never run here) and driven
  by tests/sanitize/abi_driver.c through paths that return before any device
  work.  Leak detection is off for it: the HIP runtime it links keeps global
  state until exit.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = "/opt/rocm"
LLVM = os.path.join(ROCM, "llvm", "bin")
SAN_RT = os.path.join(ROCM, "llvm", "lib", "clang")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def _clean(r):
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text and "LeakSanitizer" not in text, text


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-ffp-contract=off", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "bl_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="3"))
    _clean(r)
    assert "oracle driver done" in r.stdout


def _san_rt_dir():
    for ver in sorted(os.listdir(SAN_RT), reverse=True):
        d = os.path.join(SAN_RT, ver, "lib", "linux")
        if os.path.exists(os.path.join(d, "libclang_rt.asan-x86_64.so")):
            return d
    return None


@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "bin", "hipcc")), reason="hipcc not installed")
def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2002_08233_amd import build as hipbuild
    rt = _san_rt_dir()
    assert rt, "clang sanitizer runtime not found"
    srcs = hipbuild.SOURCES
    flags = [os.path.join(ROCM, "bin", "hipcc"), "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
             "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize=function,vptr", "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-I", os.path.join(ROOT, "include")]

    def obj(src):
        o = str(tmp_path / (src + ".o"))
        _run(flags + ["-c", os.path.join(ROOT, "paper_2002_08233_amd", "csrc", src), "-o", o])
        return o

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(obj, srcs))
    lib = str(tmp_path / "libbl_san.so")
    _run([os.path.join(LLVM, "clang++"), "-shared", "-fPIC", "-fsanitize=address,undefined",
          "-fno-sanitize=function,vptr", "-shared-libsan", "-o", lib] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    exe = str(tmp_path / "abi_driver")
    _run([os.path.join(LLVM, "clang"), "-g", "-fsanitize=address,undefined", "-shared-libsan",
          "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "abi_driver.c"), lib,
          "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + rt, "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    _clean(r)
    assert "abi driver done" in r.stdout
