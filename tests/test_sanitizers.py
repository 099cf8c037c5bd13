"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code.

Two C drivers run under the sanitizers on a machine without a GPU:

* ``oracle_sanitize_driver.c`` links the oracle's C source and runs it over
  every schedule variant, both sign modes, its refusals and its helpers;
* ``abi_sanitize_driver.c`` links the library's host sources (the device part
  of ``pa_kernels.hip`` is built normally, its host part with the sanitizers)
  and drives the C ABI's validation, planning, table, checkpoint, batch and
  pool-admission paths, none of which launches a kernel.

A sanitizer report aborts the driver, so the test only checks the exit status
and the closing line. Leak detection is off for the library driver: the HIP
runtime keeps allocations until exit.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2510_21105_amd" / "csrc"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HOST_SAN = []
for flag in ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer"]:
    HOST_SAN += ["-Xarch_host", flag]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_san"
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", *SAN, "-I", str(ROOT / "oracle"),
          str(ROOT / "tests" / "oracle_sanitize_driver.c"), str(ROOT / "oracle" / "pa_oracle.c"),
          "-lm", "-o", str(exe)])
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([str(exe)], env=env, timeout=300)
    assert "oracle sanitizer driver ok" in r.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC) or shutil.which("gcc") is None:
        pytest.skip("hipcc or gcc not available")
    inc = ["-I", str(ROOT / "include"), "-I", str(CSRC)]
    jobs = []
    for src in ["pa_api.cpp", "pa_fused.cpp", "pa_pool.cpp"]:
        jobs.append([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", *HOST_SAN, *inc, "-c",
                     str(CSRC / src), "-o", str(tmp_path / (src + ".o"))])
    jobs.append([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN, *inc,
                 "-c", str(CSRC / "pa_kernels.hip"), "-o", str(tmp_path / "pa_kernels.o")])
    jobs.append(["gcc", "-O1", "-g", "-std=c11", *SAN, "-I", str(ROOT / "include"), "-c",
                 str(ROOT / "tests" / "abi_sanitize_driver.c"), "-o", str(tmp_path / "drv.o")])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda c: _run(c, cwd=tmp_path, timeout=600), jobs))
    exe = tmp_path / "abi_san"
    objs = [str(tmp_path / o) for o in
            ["drv.o", "pa_api.cpp.o", "pa_fused.cpp.o", "pa_pool.cpp.o", "pa_kernels.o"]]
    _run([HIPCC, "-fsanitize=address,undefined", "-fno-gpu-sanitize", *objs, "-o", str(exe)],
         cwd=tmp_path, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([str(exe)], env=env, timeout=300)
    assert "library host sanitizer driver ok" in r.stdout
