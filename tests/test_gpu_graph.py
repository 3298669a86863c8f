"""HIP graphs through the C ABI (GPU): pw_graph_capture_timestep with several
steps per graph, pw_graph_begin / pw_graph_end around arbitrary library calls,
and the argument errors of the graph entry points.  Every replay is compared
bit for bit with the same work run eagerly, with unrelated eager work and
synchronisations between replays."""
import ctypes

import pytest
import torch

import oracle
from gpu_helpers import DEV, F64_TOL, max_rel, same_bits, say
from paper_2107_13500_amd import batched as BT
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16, 64), (17, 23, 96), (40, 9, 128), (5, 3, 64), (33, 50, 64), (61, 17, 96)]


def problems(seed):
    return [inputs.make_problem(nx, ny, nz, seed + d, dx=30.0 + 4 * d) for d, (nx, ny, nz) in enumerate(SHAPES)]


def assert_same_state(a, b, where):
    for d in range(len(a.fields)):
        for f, (x, y) in enumerate(zip(a.fields[d], b.fields[d])):
            assert same_bits(x, y), "%s: domain %d array %d differs" % (where, d, f)


@pytest.mark.parametrize("storage", [B.F64, B.F32], ids=["f64", "f32"])
def test_graph_of_three_timesteps_matches_three_eager_steps(storage):
    probs = problems(1200)
    ga, eb = BT.DeviceBatch(probs, storage, DEV), BT.DeviceBatch(probs, storage, DEV)
    pa, pb = ga.plan({"chunk": 512, "seg": 16}), eb.plan({"chunk": 512, "seg": 16})
    g = ga.capture_timestep(pa, seed=5, amplitude=1e-3, nsteps=3)
    scratch = torch.randn(128, 128, device=DEV)
    for r in range(3):
        say("graph replay", r, B.DTYPE_NAMES[storage])
        g.launch()
        for _ in range(3):
            eb.timestep(pb, seed=5, amplitude=1e-3)
        scratch = scratch @ scratch.T / 128.0      # unrelated eager work between replays
        torch.cuda.synchronize()
        assert int(ga.call.item()) == 3 * (r + 1) == int(eb.call.item())
        assert_same_state(ga, eb, "replay %d" % r)
    assert pa.error_count() == 0
    if storage == B.F64:
        for d in (0, 3, len(probs) - 1):
            u, v, w = ga.host_fields(d)
            p = probs[d]
            ref = oracle.advect(u, v, w, p.coeffs.tcx, p.coeffs.tcy, *p.coeffs.arrays())
            for g_, r_ in zip(ga.host_outputs(d), ref):
                assert max_rel(g_[1:-1, 1:-1], r_[1:-1, 1:-1]) <= F64_TOL
    g.close()


def test_recorded_per_domain_launches_match_eager_launches():
    """pw_graph_begin / pw_graph_end around one pw_advect per domain on the
    recording's own stream; replays on the default stream equal the eager
    launches."""
    probs = problems(1300)
    ga, eb = BT.DeviceBatch(probs, B.F64, DEV), BT.DeviceBatch(probs, B.F64, DEV)
    plans_a, plans_b = ga.per_domain_plans(), eb.per_domain_plans()
    torch.cuda.synchronize()
    g = B.Graph.record(lambda rs: ga.advect_per_domain(plans_a, rs))
    for o in (o for bt in (ga, eb) for f in bt.fields for o in f[3:]):
        o.fill_(-9.0)                              # outputs must come from the replay (halos stay -9 in both)
    torch.cuda.synchronize()
    for r in range(2):
        g.launch()
        eb.advect_per_domain(plans_b)
        torch.cuda.synchronize()
        assert_same_state(ga, eb, "replay %d" % r)
    for d, p in enumerate(probs):
        ref = oracle.advect_problem(p)
        for g_, r_ in zip(ga.host_outputs(d), ref):
            assert max_rel(g_[1:-1, 1:-1], r_[1:-1, 1:-1]) <= F64_TOL
    g.close()


def test_graph_entry_points_reject_bad_arguments():
    l = B.lib()
    h = ctypes.c_void_p()
    assert l.pw_graph_begin(None) == -1                       # no out-pointer
    side = torch.cuda.Stream()
    assert l.pw_graph_end(side.cuda_stream, ctypes.byref(h)) == -7   # not recording
    assert l.pw_graph_end(None, ctypes.byref(h)) == -1
    rs = ctypes.c_void_p()
    assert l.pw_graph_begin(ctypes.byref(rs)) == 0 and rs.value
    assert l.pw_graph_end(rs, None) == -1                     # no out-pointer: still recording
    assert l.pw_graph_end(rs, ctypes.byref(h)) == 0           # an empty recording
    assert h.value
    assert l.pw_graph_launch(h, None) == 0
    torch.cuda.synchronize()
    assert l.pw_graph_destroy(h) == 0
    assert l.pw_graph_destroy(None) == 0
    assert l.pw_graph_launch(None, None) == -1
    batch = BT.DeviceBatch(problems(1400)[:2], B.F64, DEV)
    plan = batch.plan()
    g = ctypes.c_void_p()
    assert l.pw_graph_capture_timestep(plan.handle, 2, batch.d_args.data_ptr(), 1, batch.call.data_ptr(), 1e-3,
                                       0, ctypes.byref(g)) == -1   # nsteps < 1
    assert l.pw_graph_capture_timestep(plan.handle, 3, batch.d_args.data_ptr(), 1, batch.call.data_ptr(), 1e-3,
                                       1, ctypes.byref(g)) == -8   # ndomains differs from the plan
    assert not g.value
