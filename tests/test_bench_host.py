"""Host-side parts of bench.py that need no GPU: the committed counter summary
belongs to the kernel sources as they are (so the bench line carries measured
HBM traffic), and the one-GPU contract of --gpus."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_counter_summary_matches_the_kernel_sources():
    import bench

    vals = bench.counter_summary()
    assert vals, ("profiles/half_sweep_L65536_counters.md was taken on other kernel sources; "
                  "re-take the counter passes it lists")
    traffic = bench.measured_traffic()
    alg = 3 * (65536 * 65536 // 2) // 8
    assert alg <= traffic < 2 * alg  # every algorithmic byte moves, and not twice
    issue = bench.valu_issue(280.0)
    assert 0.5 < issue["frac_of_launch"] < 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr
    assert r.stdout == ""
