"""Robustness of the C oracle (CPU only): sanitizer builds and memory limits.

The oracle runs its queries on several POSIX threads. These tests build it
together with the stress driver `tests/oracle_stress.c` (a seeded random index
with uneven cells; every thread count must reproduce the single-thread result
bit for bit) under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer, and run the plain build under address-space limits, where an
allocation that fails must end the search with an error status, never with a
signal.
"""

import os
import resource
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "oracle_stress.c"), os.path.join(ROOT, "oracle", "fbpq_oracle.c")]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")


def _build(tmp_path, name, flags):
    exe = str(tmp_path / name)
    subprocess.check_call(["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer", *flags,
                           "-o", exe, *SRC, "-lm", "-lpthread"])
    return exe


def _run(exe, args, env=None, preexec=None):
    return subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=300,
                          env=env, preexec_fn=preexec)


@pytest.mark.parametrize("args", [(1, 5000, 16, 3000, 4), (2, 40, 16, 100, 8), (300, 200000, 64, 6000, 8)])
def test_oracle_asan_ubsan(tmp_path, args):
    exe = _build(tmp_path, "stress_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    r = _run(exe, args, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle_stress ok" in r.stdout


def test_oracle_tsan(tmp_path):
    exe = _build(tmp_path, "stress_tsan", ["-fsanitize=thread"])
    r = _run(exe, (300, 100000, 48, 5000, 8), env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    if r.returncode != 0 and "FATAL: ThreadSanitizer" in r.stderr and "WARNING" not in r.stderr:
        pytest.skip("ThreadSanitizer cannot run in this environment: " + r.stderr.strip()[:200])
    assert r.returncode == 0, r.stdout + r.stderr


def test_oracle_address_space_limits(tmp_path):
    """Under an address-space cap the search returns an error or the right
    answer; an exit by signal would be a crash."""
    exe = _build(tmp_path, "stress_plain", [])
    ok = 0
    for cap_mib in (64, 96, 128, 192, 256, 384, 1024):
        cap = cap_mib << 20

        def limit(cap=cap):
            resource.setrlimit(resource.RLIMIT_AS, (cap, cap))

        r = _run(exe, (1024, 300000, 32, 20000, 16), preexec=limit)
        assert r.returncode in (0, 1, 2), f"cap {cap_mib} MiB: exit {r.returncode}\n{r.stderr}"
        ok += r.returncode == 0
    assert ok >= 1, "no cap was large enough for the search"
