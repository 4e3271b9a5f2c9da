"""bench.py refuses what it does not run, before touching a GPU: more than
one GPU or rank, and mode combinations that exclude each other."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=e,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    p = _run(["--gpus", "2"])
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_more_than_one_rank_is_refused():
    p = _run([], env={"WORLD_SIZE": "2"})
    assert p.returncode == 2 and "WORLD_SIZE" in p.stderr


@pytest.mark.parametrize("args", [["--folded", "--backward"], ["--spatial", "0.95", "--plain"],
                                  ["--material-edit", "--folded"], ["--material-edit", "--backward"]])
def test_exclusive_modes_are_refused(args):
    p = _run(args)
    assert p.returncode == 2 and "excludes" in p.stderr, p.stderr
