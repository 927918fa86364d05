"""The serving loop (csrc/pf_server.cpp) on the CPU against a host-only
stand-in of the filter ABI it calls (tests/server_mock/mock_abi.cpp): every
observation of N streams submitted at once, without pacing, completions out
of order across ticks; built with AddressSanitizer and UBSan (and with
ThreadSanitizer where the LLVM toolchain is present).  Each run must end with
every step completed and every stream closed, and no sanitizer report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "server_mock", "mock_abi.cpp"),
       os.path.join(ROOT, "paper_1411_1702_amd", "csrc", "pf_server.cpp")]
INC = os.path.join(ROOT, "include")


def _build(tmp_path, cxx, flags, name):
    exe = str(tmp_path / name)
    r = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-I", INC, *flags, "-o", exe, *SRC, "-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, n, env=None):
    r = subprocess.run([exe, str(n)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout[-500:], r.stderr[-3000:])
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    fields = dict(zip(r.stdout.split()[::2], map(int, r.stdout.split()[1::2])))
    # 70% of the streams observe 25 times, 30% 50 times (stream k: k % 10 < 7)
    want = sum(25 if k % 10 < 7 else 50 for k in range(n))
    assert fields["completed"] == want and fields["skipped"] == 0, fields
    assert fields["closed"] == n, fields


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_server_unpaced_asan(tmp_path):
    exe = _build(tmp_path, "g++", ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"], "srv_asan")
    for n in (50, 500):
        _run(exe, n)


LLVM_CXX = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(LLVM_CXX), reason="no LLVM toolchain for ThreadSanitizer")
def test_server_unpaced_tsan(tmp_path):
    # LLVM's ThreadSanitizer (GCC 11's does not intercept the clock-based
    # condition-variable wait libstdc++ uses, and reports false races)
    exe = _build(tmp_path, LLVM_CXX, ["-fsanitize=thread"], "srv_tsan")
    for n in (50, 500):
        _run(exe, n)
