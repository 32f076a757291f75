"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host part of
the library (host objects only: the layout builder, the ordering and the
host-only C entry points) and of the CPU oracle, each driven over seeded
random and malformed inputs (tests/sanitize/*_driver.*).  The host driver also
makes the n-th host allocation of a conversion fail, for every n until the
conversion gets through: each failing call must return RGCSR_ENOMEM, and
LeakSanitizer must find no leak when the driver exits."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1012_2270_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)} -> {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_library_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_asan")
    srcs = [os.path.join(CSRC, f) for f in ("host_layout.cpp", "ordering.cpp", "abi_host.cpp", "tile_layout.cpp",
                                             "panel_layout.cpp")]
    _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), *srcs,
          os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", exe])
    r = _run([exe], env=ENV, timeout=600)
    assert "each returned RGCSR_ENOMEM" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off", os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV, timeout=600)
    assert "failures: 0" in r.stdout
