"""The bench's command-line contract on the host: more than one GPU is
refused with a message (the path needs no collective and the measurement
is of one GPU), and the help lists the options the measurements use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2", "--no-cpu-baseline")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_measurement_options():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--form", "--start-level", "--chain-rule", "--triple",
                "--latlong", "--nnz", "--serial", "--copy-calibration"):
        assert opt in r.stdout, opt
