"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): every source is compiled with the sanitizers on its host side
(device code unchanged), linked with tests/asan/abi_host_check.c, and run.
The checker exercises the host-only paths of the C ABI: argument
validation and its messages, the default options, and the footprint
computation over Poisson, heat and Navier-Stokes shapes and every solver and
product precision. A sanitizer report or a failed check fails the test."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_21404_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                                reason="hipcc / clang not installed")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_host_code_under_asan_ubsan(tmp_path):
    sources = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-Wno-unused-value", *SAN,
             "-Xarch_host", "-fno-omit-frame-pointer"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(8, len(sources))) as ex:
        objs = list(ex.map(compile_one, sources))
    check_o = str(tmp_path / "abi_host_check.o")
    _run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(ROOT, "tests", "asan", "abi_host_check.c"), "-o", check_o])
    exe = str(tmp_path / "abi_host_check")
    _run([HIPCC, "--offload-arch=gfx950", *SAN, check_o, *objs, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert r.stdout.startswith("ok "), out
    assert int(r.stdout.split()[1]) > 200
    shutil.rmtree(tmp_path, ignore_errors=True)
