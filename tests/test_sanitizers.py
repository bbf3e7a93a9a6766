"""The oracle (oracle/he_oracle.c) and libhe's host arithmetic (csrc/host.cpp)
built with AddressSanitizer and UndefinedBehaviorSanitizer and run on the CPU
through the programs in tests/sanitize/: every exported routine over the ring
degrees and parameters used, with edge and refused inputs.  Host code only:
the HIP build is host-only (no device code is compiled), and the sanitizer
flags are host-side flags."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]


def _run(cmd, exe):
    _build(cmd)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])


def _oracle_cmd(exe, *extra):
    return ["gcc", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all", "-ffp-contract=off", "-Wall", *extra, "-o", exe,
            os.path.join(HERE, "sanitize", "oracle_san.c")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(_oracle_cmd(exe), exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_planted_overread_is_reported(tmp_path):
    """The same driver with one planted read past a buffer: the build reports it."""
    exe = str(tmp_path / "oracle_san_planted")
    _build(_oracle_cmd(exe, "-DPLANT_OVERREAD"))
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    # UBSan's object-size check or ASan's shadow check, whichever sees it first
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or "insufficient space" in r.stderr)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_host_arithmetic_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_2006_10091_amd", "csrc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
    _run([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-g", "-ffp-contract=off",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", csrc] + san +
         [os.path.join(HERE, "sanitize", "host_san.cpp"), os.path.join(csrc, "host.cpp"), "-o", exe], exe)
