"""Host-side checks of the benchmark script: the driver's command line
parses, and the graph schedule times exactly the requested number of steps
for any --steps (no GPU needed)."""
import subprocess
import sys
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_driver_argv_parses():
    a = bench.parse(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup) == (1, 20, 5)
    plan = bench.graph_schedule(a.steps)
    assert plan == [(20, 1)]
    assert sum(n * r for n, r in plan) == 20


@pytest.mark.parametrize("K", [1, 7, 20, 49, 50, 51, 99, 100, 137, 1000, 1001])
def test_graph_schedule_covers_exactly_K(K):
    plan = bench.graph_schedule(K)
    assert sum(n * r for n, r in plan) == K
    assert all(n >= 1 and r >= 1 for n, r in plan)
    assert plan[0][0] == min(50, K)
    assert len(plan) <= 2


def test_graph_schedule_rejects_zero_steps():
    with pytest.raises(ValueError):
        bench.graph_schedule(0)


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_host_info_fields():
    h = bench.host_info()
    assert h["nproc"] >= 1 and h["logical_cpus"] >= 1
