"""bench.py's command-line contract, on the host: one GPU only, and the report flags."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=300)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_flags_are_listed():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--no-cpu", "--no-extras", "--paper-protocol"):
        assert flag in r.stdout


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU may be visible here")
def test_no_gpu_is_an_error_not_a_fallback():
    r = _run("--paper-protocol")
    assert r.returncode == 1
    assert json.loads(r.stdout.strip().splitlines()[-1]) == {"error": "no GPU visible"}
