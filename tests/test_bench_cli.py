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


def test_cpu_baseline_reports_the_timed_outputs_error():
    """The bench's accuracy clause on the host: the checker runs in the
    worker pool on the stored inputs it is given, and the reported rel-L2 is
    that of the given device output against it (0 for the checker's own
    result, the planted relative error for a scaled one)."""
    import numpy as np
    sys.path.insert(0, ROOT)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import bench
    from cases import build_case, reference, workload
    # as many frames as sampled vertices: only the per-vertex arguments split
    case = build_case(workload(61, 8, 40, 12, 32, nframes=12))
    inputs = (case["light_idx"], case["light_val"], 8, bench.PerVertex(case["vert_rot"]),
              case["frame_rot"], bench.PerVertex(case["t_idx"]), bench.PerVertex(case["t_val"]))
    ref = reference(case)
    pool = bench.start_cpu_pool(2)
    try:
        base, err, got_ref = bench.cpu_baseline(pool, 2, inputs, ref, "test")
        assert err == 0.0 and np.array_equal(got_ref, ref)
        assert base["cores"] == 2 and base["kind"] == "oracle" and base["value"] > 0
        _, err, _ = bench.cpu_baseline(pool, 2, inputs, ref * (1 + 3e-6), "test")
        assert abs(err - 3e-6) < 1e-9
    finally:
        pool.close()
        pool.join()
    vids = bench.accuracy_sample(50000, 64, 4096)
    assert len(vids) == 64 and np.all(np.diff(vids) > 0)
    assert len(bench.accuracy_sample(50000, 1, 4096)) == 4096
