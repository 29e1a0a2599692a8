"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host front end (argument validation, slab decomposition,
  detector row bands, the projection matrix, tile sizing: fdk_api.cpp,
  tiles.cpp and the host halves of the .hip files) is rebuilt with the
  sanitizers on the host side only (-Xarch_host; device code is unchanged)
  and the C-ABI tests run against it in a child process that preloads the
  sanitizer runtime.
* The oracle (oracle.c) is rebuilt with gcc's sanitizers and its pinning
  tests run against it the same way.
* The tile-bound checker (the kernels' brick setup and FP32 column
  arithmetic built for the host) runs as a sanitized executable.

Any sanitizer report aborts the child (halt_on_error), which fails the test.
"""
import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_02724_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer"]
HIP_FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "--offload-arch=gfx950", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
             "-fvisibility=hidden"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def _child_pytest(module, attr, libpath, tests, preload):
    """Run pytest on `tests` in a child process whose `module.attr` (the
    library path the ctypes loader opens) points at the sanitized build."""
    code = (f"import sys; sys.path.insert(0, {ROOT!r}); import {module} as m; "
            f"m.{attr} = {libpath!r}; m._lib = None; import pytest; "
            f"rc = pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '-m', 'not gpu'] + "
            f"{tests!r}); "
            f"assert {libpath!r} in open('/proc/self/maps').read(), 'sanitized library not loaded'; "
            f"sys.exit(rc)")
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       cwd=ROOT, timeout=600)
    assert r.returncode == 0, f"child failed ({r.returncode}):\n{r.stdout[-6000:]}\n{r.stderr[-6000:]}"
    return r.stdout


def test_front_end_under_asan_ubsan(tmp_path):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.cpp")) + glob.glob(os.path.join(CSRC, "*.hip")))

    def compile_one(src):
        obj = tmp_path / (os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([HIPCC, *HIP_FLAGS, *SAN_HOST, *lang, "-c", src, "-o", str(obj)])
        return str(obj)

    with ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libfdk_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan", *SAN_HOST[:4],
          "-o", lib, *objs])
    rt = _run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"]).stdout.strip()
    out = _child_pytest("paper_1909_02724_amd", "LIB_PATH", lib,
                        ["tests/test_abi.py"], rt)
    assert " passed" in out and "failed" not in out, out


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", lib,
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    rt = ":".join(_run(["gcc", f"-print-file-name={n}"]).stdout.strip()
                  for n in ("libasan.so", "libubsan.so"))
    out = _child_pytest("oracle", "_LIB", lib,
                        ["tests/test_oracle_bp.py", "tests/test_oracle_geometry.py",
                         "tests/test_oracle_sirt.py", "tests/test_oracle_phantom_filter.py",
                         "tests/test_synth_noise.py"], rt)
    assert " passed" in out and "failed" not in out, out


def test_tile_checker_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "tile_bounds_check_san")
    _run([HIPCC, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "--cuda-host-only", *SAN_HOST,
          "-x", "hip", os.path.join(ROOT, "tests", "tile_bounds_check.cpp"),
          "-x", "c++", os.path.join(CSRC, "tiles.cpp"), "-o", exe])
    r = subprocess.run([exe, "7", "300"], capture_output=True, text=True,
                       env=dict(os.environ, **SAN_ENV), timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "col_viol=0 row_viol=0" in r.stdout, r.stdout
