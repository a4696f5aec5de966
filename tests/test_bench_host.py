"""Host logic of bench.py, without a GPU: the one-GPU guard, the field-error and bound
bookkeeping of the mixed form, and the counter summaries that the roofline reads."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N_CHANNEL = 400 * 500 * 2 * 200     # live particles of the channel workload the counters were taken on


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _stats(n, rng):
    s = rng.uniform(0.5, 2.0, size=(n, 13))
    s[:5] = np.nan                      # nodes without particles
    return s


def test_field_errors_are_weighted_relative_norms():
    rng = np.random.default_rng(5)
    ref = _stats(200, rng)
    assert all(v == 0.0 for v in bench.field_errors(ref.copy(), ref).values())
    # a uniform relative change of one field gives that relative error for it alone
    s = ref.copy()
    s[:, 4] *= 1 + 3e-6
    err = bench.field_errors(s, ref)
    assert abs(err["omega"] - 3e-6) < 1e-12
    assert all(err[k] == 0.0 for k in ("W", "U", "psi", "R", "psi_var"))
    # off-diagonal stresses count twice in the tensor norm: the same absolute change on
    # u1u2 weighs sqrt(2) times what it weighs on u1u1
    a, b = ref.copy(), ref.copy()
    a[:, 6] += 1e-3
    b[:, 9] += 1e-3
    assert abs(bench.field_errors(b, ref)["R"] / bench.field_errors(a, ref)["R"] - np.sqrt(2.0)) < 1e-9


def test_bounds_list_exactly_the_fields_over_them():
    err = {"W": 1e-6, "U": 2e-5, "omega": 1e-5, "psi": 5e-5, "R": 2e-4, "psi_var": 1e-9}
    out = bench.with_bounds(dict(err))
    assert out["misses"] == ["R", "U"]           # a value equal to its bound meets it
    assert out["bounds"]["omega"] == 1e-5 and out["bounds"]["R"] == 1e-4


def test_counter_summaries_are_consistent():
    """The committed counter summary, when it matches the kernel source, gives traffic per
    launch at least the kernels' algorithmic bytes and below three times them, and the
    particle loop's average time agrees with the kernel trace of the same source."""
    for kernel in ("advance", "element_pass", "scatter"):
        t = bench.counter_traffic(kernel, True)
        if t is None:          # kernels changed since the counters were taken
            continue
        alg = bench.BYTES_PER_PARTICLE[kernel] * N_CHANNEL
        assert 0.9 * alg <= t <= 3.0 * alg, (kernel, t / alg)
    ms = bench.measured("advance", "avg_ms", True)
    trace = os.path.join(ROOT, "profiles", "kernel_trace_channel_large.txt")
    if ms is not None and os.path.exists(trace):
        lines = open(trace).read().splitlines()
        sha = [ln for ln in lines if ln.startswith("kernels.hip sha256 prefix:")]
        if sha and sha[0] in open(bench.COUNTERS).read():
            row = [ln.split() for ln in lines if ln.startswith("k_advance<double, false>")][0]
            assert abs(float(row[-2]) - ms) / ms < 0.1


def test_counter_summary_of_another_source_is_not_used(tmp_path):
    p = tmp_path / "c.txt"
    p.write_text("kernels.hip sha256 prefix: 0000000000000000\nmeasure k_advance read_bytes_per_launch 1\n")
    assert bench.measured("advance", "read_bytes_per_launch", True, str(p)) is None
    assert bench.measured("advance", "read_bytes_per_launch", False) is None
