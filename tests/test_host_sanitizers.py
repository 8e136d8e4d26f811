"""Host code of libtomo (tomo_api.cpp, unet_api.cpp, pipeline.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer instrumentation on its host side only (the device code is as in
the library), linked with the library's kernel objects, and run through every ABI validation
path that needs no GPU (tests/sanitize_abi.cpp)."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_28756_amd", "csrc")
LIBDIR = os.path.join(ROOT, "paper_2603_28756_amd", "lib")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
# sanitizer flags reach the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout[-3000:]}\n{res.stderr[-3000:]}"
    return res


def test_abi_host_paths_under_asan_and_ubsan(tmp_path):
    kernel_objs = [o for o in glob.glob(os.path.join(LIBDIR, "*_kernels.hip.o"))]
    if not os.path.exists(HIPCC) or not os.path.exists(CLANG) or len(kernel_objs) < 4:
        pytest.skip("needs hipcc, clang++ and the library's kernel objects (run the build first)")
    inc = os.path.join(ROOT, "include")
    objs = []
    for src in ("tomo_api.cpp", "unet_api.cpp", "pipeline.cpp"):
        o = str(tmp_path / (src + ".o"))
        _run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", inc, *HOST_SAN, "-x", "hip", "-c",
              os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = str(tmp_path / "sanitize_abi.o")
    _run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-I", inc, "-c", os.path.join(ROOT, "tests", "sanitize_abi.cpp"), "-o", drv])
    exe = str(tmp_path / "sanitize_abi")
    _run([CLANG, "-fsanitize=address,undefined", "-o", exe, drv, *objs, *kernel_objs,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = _run([exe], env=env, timeout=300)
    assert "sanitized host checks passed" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
