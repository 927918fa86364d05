"""The oracle's CPU pins run once more on a build of the oracle with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc), in a child process
that preloads the sanitizer runtimes: any out-of-bounds access, use after
free or undefined operation the pins reach aborts the child."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    lib = str(tmp_path / "liboracle_san.so")
    O.compile_to(O.SRC, lib, extra=["-O1", "-g", "-fno-omit-frame-pointer",
                                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    files = [f for f in files if not f.endswith("test_oracle_mutations.py")]
    env = dict(os.environ, PF_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu"] + files,
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-3000:]
    print(tail)
    assert res.returncode == 0, tail
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, tail
