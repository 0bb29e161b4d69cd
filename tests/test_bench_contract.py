"""Host-side checks of bench.py's command-line contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_flop_model_counts_the_pcg_iterations():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1803_10270_amd import workloads as W
    p = W.advection_ie_variable(seed=0)
    one = bench.flop_model(p, [{"sweeps": 1, "pcg_iters": 1.0}])
    more_iters = bench.flop_model(p, [{"sweeps": 1, "pcg_iters": 5.0}])
    two = bench.flop_model(p, [{"sweeps": 1, "pcg_iters": 1.0}, {"sweeps": 1, "pcg_iters": 1.0}])
    assert one > 0 and more_iters > one
    assert abs(two - 2 * one) <= 1e-9 * two
