"""bench.py's command line: refusals that need no GPU (they exit before any
device or index work)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=60)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2 and "one GPU only" in r.stderr and not r.stdout


@pytest.mark.parametrize("forms, msg", [("served", "need plain, batched or heuristic"),
                                        ("batched,foo", "unknown form")])
def test_bad_form_sets_are_refused(forms, msg):
    r = _run("--forms", forms)
    assert r.returncode == 2 and msg in r.stderr and not r.stdout
