"""Host code under AddressSanitizer and UBSan (CPU only): the C-ABI layer of the
library (argument checks, workspace carving, launch sequencing), linked with
launcher stand-ins that check every workspace range they are handed, and the C
oracle on small fields. Both are built with g++/gcc (no device code)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_api_host_layer_under_sanitizers(tmp_path):
    exe = str(tmp_path / "api_driver")
    subprocess.check_call(
        ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__=1", "-I/opt/rocm/include",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2208_12569_amd", "csrc"),
         os.path.join(ROOT, "paper_2208_12569_amd", "csrc", "api.cpp"),
         os.path.join(HERE, "api_stubs.cpp"), os.path.join(HERE, "api_driver.cpp"), "-o", exe])
    out = _run(exe)
    assert "0 failures" in out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(
        ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", *SAN, "-Wno-unknown-pragmas",
         "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "fq_oracle.c"),
         os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"])
    out = _run(exe)
    assert "0 failures" in out
