"""bench.py's command-line contract on the CPU: one GPU only (a clear refusal
for more, before anything touches a device) and the documented flags."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True, timeout=120, env=e)


def test_more_than_one_gpu_is_refused():
    r = run(["--gpus", "2"])
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    r = run([], env={"WORLD_SIZE": "2"})
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_flags_are_documented():
    r = run(["--help"])
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--no-cpu-baseline", "--no-batched", "--no-serving", "--no-adversarial",
                 "--no-smallest", "--no-by-k", "--no-host", "--copy-calibration", "--delegate-vector"):
        assert flag in r.stdout, flag
