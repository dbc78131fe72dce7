"""AddressSanitizer and UndefinedBehaviorSanitizer run of the C ABI's host code.

The library is rebuilt with both sanitizers on its host code (device code is
compiled as usual and never launched), a small C driver (tests/abi_sanitize.c)
is linked against it and calls every entry point with invalid arguments and the
setup entry point with valid ones: the argument checks, the scans over the
level-set and label arrays (allocated with exactly the documented size) and the
error returns must run without a sanitizer report or leak, and every call must
return the documented status.  No GPU is used: with no device present, valid
arguments end in XFFT_EDEVICE after the validation.
"""

import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_02172_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


def _asan_runtime_dir():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return os.path.dirname(sorted(hits)[-1]) if hits else None


@pytest.mark.slow
def test_abi_validation_under_host_sanitizers(tmp_path):
    rt = _asan_runtime_dir()
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG) and rt):
        pytest.skip("hipcc, clang or the clang sanitizer runtime not found")
    from paper_2601_02172_amd.build import SOURCES
    # sanitizers on the host side only: each -fsanitize= follows -Xarch_host
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([HIPCC] + common + san + ["-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    lib = str(tmp_path / "libxfft_asan.so")
    r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + san[:4] +
                       ["-shared-libsan", "-o", lib] + objs, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    # the library really is instrumented
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout if shutil.which("nm") else ""
    if nm:
        assert "__asan_report" in nm and "__ubsan_handle" in nm
    exe = str(tmp_path / "abi_sanitize")
    r = subprocess.run([CLANG, "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-shared-libsan", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "abi_sanitize.c"), "-o", exe, "-L", str(tmp_path),
                        "-lxfft_asan", f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{rt}", "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
