"""The benchmark's command line on the CPU: the checks that run before it
touches a GPU (the one-GPU limit, section names)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=ROOT, env=e, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_world_size_above_one_is_refused():
    r = _bench(env={"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_unknown_section_is_refused_with_the_list():
    r = _bench("--only", "compress,nosuch")
    assert r.returncode == 2
    assert "nosuch" in r.stderr and "transpose" in r.stderr and "half" in r.stderr
