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


def test_step_roofline_bounds_and_fractions():
    """Whole-step bounds from their closed forms: 2 (2 I m RR + m RR^2) FLOP
    at 157.3 TFLOP/s for the 400^3 step, 9.4 MB at 8 TB/s for the batch, and
    2 * 64^4 * 25 FLOP at 78.6 TFLOP/s for the optimal law; each fraction is
    bound / measured."""
    main = {"ms_per_step": 0.05}
    plain = {"f32": {"us_per_step": 25.0}}
    batched = {"ms_per_batch_step": 0.1}
    laws4 = {"laws": {"O": {"us_per_step": 100.0}}}
    out = bench.step_roofline(main, plain, batched, laws4, 400, 10, 4096)
    c3 = 2 * (2 * 400 * 4096 * 100 + 4096 * 100 * 100) / 157.3e12 * 1e6
    assert out["scaled_fp32"]["bound_us"] == pytest.approx(c3, abs=1e-3)
    assert out["scaled_fp32"]["frac"] == pytest.approx(c3 / 50.0, abs=1e-4)
    assert out["plain_fp32"]["frac"] == pytest.approx(c3 / 25.0, abs=1e-4)
    assert out["batched_64"]["bound_us"] == pytest.approx(9.4e6 / 8e12 * 1e6, abs=1e-3)
    assert out["batched_64"]["frac"] == pytest.approx(1.175 / 100.0, abs=1e-4)
    o = 2 * 64 ** 4 * 25 / 78.6e12 * 1e6
    assert out["optimal_law_order4"]["bound_us"] == pytest.approx(o, abs=1e-3)
    assert out["optimal_law_order4"]["frac"] == pytest.approx(o / 100.0, abs=1e-4)
    assert set(bench.step_roofline(main, None, None, None, 400, 10, 4096)) == {"scaled_fp32"}
