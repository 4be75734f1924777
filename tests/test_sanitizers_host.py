"""The oracle's C source and the host builds of the solver's headers (the FP64
polish, the chunked polish with its contact-parallel team, the cone barrier
polish, the coarse-stage query) rebuilt with AddressSanitizer and
UndefinedBehaviorSanitizer and run through a selection of their CPU tests in a
child pytest: any out-of-bounds access, use after free, signed overflow,
misaligned or null access, or invalid shift ends the child with a report."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SELECTION = [
    "test_polish_host.py",
    "test_gpolish_host.py::test_chunked_polish_reaches_the_minimiser[1-1-12]",
    "test_gpolish_host.py::test_chunked_polish_reaches_the_minimiser[12-3-12]",
    "test_gpolish_host.py::test_group_factor_in_memory_matches_the_register_form[3]",
    "test_cone_host.py::test_projection_matches_closest_point_of_triangle",
    "test_cone_host.py::test_polish_matches_oracle[kernel_schedule-2.0-cold]",
    "test_hand_host.py",
    "test_oracle_kkt_and_cases.py",
    "test_oracle_bruteforce.py",
    "test_oracle_sensitivity.py",
    "test_oracle_frame_and_G.py",
    "test_oracle_golden.py",
    "test_oracle_admm_kkt.py",
]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=%s" % name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    env = dict(os.environ)
    env.update({
        "BODEX_SANITIZE": "1",
        "ORACLE_LIB": str(tmp_path / "liboracle_san.so"),
        "ORACLE_CFLAGS": "-fsanitize=address,undefined -fno-sanitize-recover=all -fno-omit-frame-pointer -O1 -g",
        "LD_PRELOAD": asan,
        # the interpreter's own allocations are not instrumented: leaks there
        # are not this code's
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           *[os.path.join(HERE, s) for s in SELECTION]]
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (p.stdout + p.stderr)[-6000:]
    assert p.returncode == 0, "sanitizer run failed (exit %d):\n%s" % (p.returncode, tail)
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
    print(p.stdout.strip().splitlines()[-1])
