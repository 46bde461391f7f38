"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and exit status 2, before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_help_lists_the_contract_flags():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup"):
        assert flag in r.stdout


def test_cpu_baseline_budget_fit():
    """The CPU baselines' sample sizing grows the sample until one run takes a
    quarter of the budget or reaches the cap, and returns that last run."""
    sys.path.insert(0, ROOT)
    import bench
    calls = []

    def run(n):
        calls.append(n)
        return n * 1e-3 + 0.01, n        # a fixed cost plus a per-sample cost

    n, t, res = bench._fit_to_budget(run, 4.0, 16, 10**9)
    assert t >= 1.0 and res == n and calls[-1] == n and calls == sorted(calls)
    n, t, res = bench._fit_to_budget(run, 4.0, 16, 100)      # the cap ends it first
    assert n == 100 and t < 1.0
    n, t, res = bench._fit_to_budget(run, 4.0, 5000, 10**9)  # the first run is enough
    assert n == 5000 and len([c for c in calls if c == 5000]) == 1
