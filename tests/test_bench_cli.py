"""bench.py's host-side contract (CPU only): the one-GPU limit, and the
committed rocprofv3 traffic profile matching the current kernel build."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_traffic_profile_matches_the_kernel_build():
    """bench.py reports roofline.traffic only while the profile under
    profiles/ was taken from the current kernel sources and launch shape."""
    import bench
    t = bench.measured_traffic("pw_march_f64_pw2048", 512, 128)
    assert t is not None, "profiles/pw_march_f64_pw2048.json is stale: profile the current kernels again"
    assert 12_897_492_992 <= t < 1.1 * 12_897_492_992
