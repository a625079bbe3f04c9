"""The benchmark's command line on the CPU: it measures one GPU only and
refuses a multi-GPU request before touching a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=e,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)


def test_multi_gpu_request_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)
    assert not r.stdout.lstrip().startswith("{")  # no result line


def test_multi_rank_launch_is_refused():
    r = _run(["--gpus", "1"], env={"WORLD_SIZE": "2"})
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)
