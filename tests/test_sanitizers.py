"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU-side
code (CPU only, no GPU calls): the oracle, driven on small and edge-case
inputs, and the host half of the library's C ABI (argument validation, the
tuning table's JSON reader with malformed files, the code-stream header)."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1404_0774_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
# the library's own source list
from paper_1404_0774_amd.build import SOURCES as _LIB_SOURCES  # noqa: E402
SOURCES = [os.path.splitext(f)[0] for f in _LIB_SOURCES]
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
         os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "fic_oracle.c"),
         "-lm", "-o", exe])
    r = run([exe], env=SAN_ENV)
    assert "oracle driver ok" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no hipcc")
def test_host_abi_under_asan_ubsan(tmp_path):
    # the whole library, sanitizers on the host pass only (each -fsanitize
    # is given to the host pass; device code is built as usual)
    def compile_one(name):
        obj = str(tmp_path / f"{name}.o")
        run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-c", os.path.join(CSRC, f"{name}.hip"), "-o", obj])
        return obj
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv = str(tmp_path / "abi_driver.o")
    run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "abi_driver")
    run([CLANG, "--hip-link", "--offload-arch=gfx950", "-fsanitize=address,undefined",
         "-fno-gpu-sanitize", drv, *objs,
         "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    # the HIP runtime keeps allocations until exit: leak checking is for the oracle
    env = dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=0")
    jdir = tmp_path / "json"
    jdir.mkdir()
    r = run([exe, str(jdir)], env=env)
    assert "abi driver ok" in r.stdout
