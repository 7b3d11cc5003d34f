"""bench.py's command line on the host: more than one GPU is refused before
anything touches a device, with a message and a non-zero status."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          env=e, capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        r = _run(["--gpus", n, "--steps", "1", "--warmup", "0"])
        assert r.returncode == 2
        assert "exactly one GPU" in r.stderr and ("--gpus %s" % n) in r.stderr
        assert r.stdout == ""


def test_several_ranks_are_refused():
    r = _run(["--steps", "1"], env={"WORLD_SIZE": "2"})
    assert r.returncode == 2 and "exactly one GPU" in r.stderr
