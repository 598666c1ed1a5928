"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only; GPU code is never built with a sanitizer).

* tests/sanitize/cpu_check.c: the oracle (every variant, queries, decode) and
  the multicore pwt / dd comparator on many small seeded inputs, pwt and dd
  compared with the oracle word by word (gcc, OpenMP).
* tests/sanitize/host_check.cpp: the library's host planning code (layouts,
  batch / buffered / multiary / Huffman plans, tuning table, argument checks)
  through the C ABI entry points that touch no device; the HIP sources are
  compiled with the sanitizers on their host side only.
"""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1610_05994_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_and_multicore_comparator_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "cpu_check")
        _run(["gcc", "-std=c99", "-O1", "-g", *SAN_FLAGS, "-fopenmp", "-o", exe,
              os.path.join(ROOT, "oracle", "wt_oracle.c"),
              os.path.join(ROOT, "paper_1610_05994_amd", "cpu", "wt_cpu.c"),
              os.path.join(SAN, "cpu_check.c")])
        env = dict(os.environ, OMP_NUM_THREADS="3", ASAN_OPTIONS="detect_leaks=1")
        r = _run([exe], env=env, timeout=600)
        assert "cpu checks: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_code_under_sanitizers():
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    with tempfile.TemporaryDirectory() as d:
        inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

        def obj(src):
            out = os.path.join(d, src.replace(".hip", ".o"))
            _run([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-Xarch_host", SAN_FLAGS[0], "-Xarch_host", SAN_FLAGS[1], *inc, "-c",
                  os.path.join(CSRC, src), "-o", out])
            return out

        with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            objs = list(ex.map(obj, srcs))
        drv = os.path.join(d, "host_check.o")
        _run([CLANG, "-std=c++17", "-O1", "-g", *SAN_FLAGS, *inc, "-c", os.path.join(SAN, "host_check.cpp"),
              "-o", drv])
        exe = os.path.join(d, "host_check")
        _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", SAN_FLAGS[0], *objs, drv, "-o", exe])
        r = _run([exe], timeout=600, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
        assert "host checks: ok" in r.stdout
