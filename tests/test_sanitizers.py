"""Host sanitizer runs (CPU only): the oracle's C sweeps built with gcc and
the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged), each driven through its
entry points by a small program under tests/sanitize/.  A report from either
sanitizer, or a failed check, fails the test."""

import glob
import importlib.util
import os
import shutil
import subprocess
import concurrent.futures as cf

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), res.stdout[-4000:], res.stderr[-4000:])
    return res


def _clean(res):
    text = res.stdout + res.stderr
    assert "AddressSanitizer" not in text, text[-4000:]
    assert "runtime error" not in text, text[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "stencil_oracle.c"), "-lm", "-o", exe])
    res = _run([exe], env=dict(ENV, OMP_NUM_THREADS="4"))
    _clean(res)
    assert "ok" in res.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="no hipcc")
def test_c_abi_host_code_under_asan_ubsan(tmp_path):
    spec = importlib.util.spec_from_file_location(
        "stencil_build_lib", os.path.join(ROOT, "paper_2103_09235_amd", "build_lib.py"))
    bl = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bl)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    # device code unoptimised (it is not under test and builds faster)
    flags = [f for f in bl.COMMON if f != "-O3"] + ["-O1", "-Xarch_device", "-O0"] + san
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2103_09235_amd", "csrc", "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC] + flags + ["-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "abi_driver.o")
    _run([CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
          "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "abi_driver.cpp"),
          "-o", drv])
    exe = str(tmp_path / "abi_driver")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", drv] + objs + ["-o", exe])
    res = _run([exe], env=ENV)
    _clean(res)
    assert "ok" in res.stdout
