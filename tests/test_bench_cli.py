"""bench.py's command line on the CPU: a run on more than one GPU is refused before any
device work (the evaluator is measured on one MI355X), whether asked by --gpus or by a
launcher's WORLD_SIZE."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, **env):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env={**os.environ, **env}, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""
    r = _run(["--gpus", "1"], WORLD_SIZE="4")
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_help_lists_the_leg_switches():
    r = _run(["--help"])
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--no-learned", "--no-free", "--no-free-timed", "--no-cpu"):
        assert flag in r.stdout
