"""The C oracle's tests once more against an AddressSanitizer +
UndefinedBehaviorSanitizer build of the same source (any report aborts the
run), in a child process with the sanitizer runtime preloaded; and a check
that the sanitizers are live there (an out-of-bounds write planted in the
call, not in the oracle, is caught)."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_ORACLE_TESTS = ["test_oracle_kn.py", "test_oracle_step.py", "test_oracle_ntc.py", "test_oracle_kinematics.py",
                  "test_oracle_philox.py", "test_oracle_beam_gas.py"]


def _asan_runtime():
    cands = sorted(glob.glob("/usr/lib/x86_64-linux-gnu/libasan.so.*")) + sorted(glob.glob("/usr/lib64/libasan.so.*"))
    return cands[0] if cands else None


@pytest.fixture(scope="module")
def sanitized_env():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime on this host")
    sys.path.insert(0, ROOT)
    from oracle import build

    lib = build.build(sanitized=True)
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "halt_on_error=1",
                "CS_ORACLE_LIB": lib})
    return env


@pytest.mark.slow
def test_c_oracle_tests_pass_under_sanitizers(sanitized_env):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", t) for t in C_ORACLE_TESTS]],
                       cwd=ROOT, env=sanitized_env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr


def test_sanitizers_are_live(sanitized_env):
    code = ("import numpy as np, oracle\n"
            "assert oracle._LIB_PATH.endswith('liboracle_sanitized.so')\n"
            "out = np.empty(10, dtype=np.int64)\n"
            "oracle.lib().oracle_shuffle_all(100, 0, 0, 0, out.ctypes.data)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=sanitized_env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]
