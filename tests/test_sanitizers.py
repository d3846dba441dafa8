"""Sanitizer builds on the CPU (no GPU needed):

* the join oracle built with AddressSanitizer + UndefinedBehaviorSanitizer and
  driven by tests/sanitize/oracle_selftest.c (every entry point, duplicates,
  negative keys, empty sides, one and several sort threads, cross-checks of the
  three join functions);
* the library's host code (the host side of every .hip file; hipcc takes each
  -fsanitize flag after -Xarch_host, so device code is built as usual) driven
  by tests/sanitize/host_selftest.c through the C ABI: planning under every
  selector, workspace sizing of every variant over a sweep of sizes and knobs,
  the argument checks that precede any GPU work, selector and batch host paths.

ThreadSanitizer is not used: the oracle's threads are OpenMP, whose runtime
(libgomp) is not TSan-instrumented, so TSan reports the runtime's own reduction
and barrier traffic as races."""
import concurrent.futures as cf
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          "-fopenmp", "-std=c11", "-o", exe, os.path.join(SAN, "oracle_selftest.c"),
          os.path.join(ROOT, "oracle", "eiger_oracle.c")])
    r = _run([exe], env=ENV, timeout=600)
    assert "oracle selftest ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_code_under_asan_ubsan(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
             "-I", os.path.join(ROOT, "paper_2607_04489_amd", "csrc"),
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2607_04489_amd", "csrc", "*.hip")))

    def build(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *flags, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(build, srcs))
    exe = str(tmp_path / "host_san")
    _run([HIPCC, "-O1", "-g", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"), *san[:4],
          "-x", "c", os.path.join(SAN, "host_selftest.c"), "-x", "none", *objs, "-o", exe])
    r = _run([exe], env=ENV, timeout=600)
    assert "host selftest ok" in r.stdout
