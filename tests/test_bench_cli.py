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
    # the default FP64 launch shapes: chunk 512, 64-plane segments on 2048 x 2048 x 64, 16 on 512 x 512 x 64
    for key, seg, algo in (("pw_march_f64_pw2048", 64, 12_897_492_992), ("pw_march_f64_pw512", 16, 808_460_288)):
        t = bench.measured_traffic(key, 512, seg)
        assert t is not None, "profiles/%s.json is stale: profile the current kernels again" % key
        assert algo <= t < 1.1 * algo


def _record(**over):
    rec = {"value": 140.0,
           "parity_f64": {"max_rel": 3.8e-16},
           "pw512": {"parity_f64": {"max_rel": 4.0e-16}},
           "precision": {"f32": {"error_vs_f64_oracle": {"max_rel": 2.1e-7}},
                         "bf16": {"error_vs_f64_oracle": {"max_rel": 8.6e-3}},
                         "f16": {"error_vs_f64_oracle": {"max_rel": 1.0e-3}},
                         "i16": {"error_vs_f64_oracle": {"max_rel": 5.1e-4}},
                         "i32": {"error_vs_f64_oracle": {"max_rel": 7.7e-9}}},
           "batched": {"f64": {"max_rel_err_sampled": 4.2e-16}, "f32": {"max_rel_err_sampled": 1.8e-7}}}
    rec.update(over)
    return rec


def test_parity_gate_passes_a_record_within_its_bounds():
    import bench
    assert bench.parity_gate(_record()) == []
    # figures that were not computed (no CPU leg) are not checked
    assert bench.parity_gate({"value": 1.0}) == []


def test_parity_gate_names_every_figure_beyond_its_bound():
    import bench
    bad = _record(parity_f64={"max_rel": 2e-12})
    bad["pw512"]["parity_f64"]["max_rel"] = float("nan")
    bad["precision"]["bf16"]["error_vs_f64_oracle"]["max_rel"] = 0.05
    bad["batched"]["f32"]["max_rel_err_sampled"] = 1e-4
    fails = bench.parity_gate(bad)
    assert len(fails) == 4
    for where in ("f64:", "pw512 f64", "storage bf16", "batched f32"):
        assert any(f.startswith(where) for f in fails), (where, fails)
