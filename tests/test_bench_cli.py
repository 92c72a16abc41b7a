"""bench.py's command line on the CPU: more than one GPU is refused with a
message before any GPU work."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=e,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")          # no JSON line


def test_world_size_above_one_is_refused():
    r = _bench(env={"WORLD_SIZE": "2"})
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
