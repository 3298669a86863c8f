"""Batched subdomains, halo fill, perturbation, graph replay and autotuner (GPU).

Each domain of a batched call must equal the oracle to 1e-12 (FP64) and be
bit-identical to a single-domain pw_advect with the same chunk and segment
shape (the batched kernel runs the same per-tile code).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import DEV, F64_TOL, max_rel, same_bits, say
from paper_2107_13500_amd import batched as BT
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

pytestmark = pytest.mark.gpu

SMALL = [(16, 16, 64), (17, 23, 96), (40, 9, 128), (5, 3, 64), (96, 31, 96), (33, 50, 64), (1, 1, 64),
         (20, 20, 128), (61, 17, 96)]


def small_problems(shapes=SMALL, seed=300):
    out = []
    for d, (nx, ny, nz) in enumerate(shapes):
        out.append(inputs.make_problem(nx, ny, nz, seed + d, dx=25.0 + 7 * d, rho0=1.1 + 0.02 * d,
                                       scale_height=6000.0 + 400 * d))
    return out


def single_outputs(batch, d, tuning):
    """pw_advect on domain d's device inputs into fresh buffers."""
    f = batch.fields[d]
    outs = [torch.zeros_like(f[0]) for _ in range(3)]
    plan = B.Plan(batch.storage, [batch.records[d].shape], tuning)
    p = batch.problems[d]
    B.advect(plan, f[0], f[1], f[2], *outs, p.coeffs.tcx, p.coeffs.tcy, *batch.tz[d],
             scales=batch.scales[d] if batch.storage in B.SCALED else None)
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("tuning", [{"chunk": 256, "seg": 8}, {"chunk": 512, "seg": 64},
                                    {"chunk": 1024, "seg": 16, "wg_per_cu": 2},
                                    {"chunk": 512, "seg": 16, "wg_per_cu": B.WG_ONE_PER_TILE}],
                         ids=["c256s8", "c512s64", "c1024s16w2", "c512s16-one-per-tile"])
def test_batched_f64_parity_and_bit_identity(tuning):
    probs = small_problems()
    batch = BT.DeviceBatch(probs, B.F64, DEV)
    plan = batch.plan(tuning)
    say("batched", tuning, plan.info())
    batch.advect(plan)
    torch.cuda.synchronize()
    assert plan.error_count() == 0
    single_t = dict(tuning, variant=B.VARIANT_MARCH)
    single_t.pop("wg_per_cu", None)
    for d, p in enumerate(probs):
        ref = oracle.advect_problem(p)
        got = batch.host_outputs(d)
        for name, g, r in zip(("su", "sv", "sw"), got, ref):
            e = max_rel(g[1:-1, 1:-1], r[1:-1, 1:-1])
            assert e <= F64_TOL, "domain %d %s: %.3e" % (d, name, e)
        for a, b in zip(batch.fields[d][3:], single_outputs(batch, d, single_t)):
            assert same_bits(a[1:-1, 1:-1], b[1:-1, 1:-1]), "domain %d differs from pw_advect" % d


@pytest.mark.parametrize("storage", [B.F32, B.BF16, B.F16, B.I16, B.I32], ids=["f32", "bf16", "f16", "i16", "i32"])
def test_batched_reduced_storage_matches_single_calls(storage):
    probs = small_problems(seed=400)
    batch = BT.DeviceBatch(probs, storage, DEV)
    tuning = {"chunk": 512, "seg": 16}
    plan = batch.plan(tuning)
    batch.advect(plan)
    torch.cuda.synchronize()
    for d in range(len(probs)):
        for a, b in zip(batch.fields[d][3:], single_outputs(batch, d, dict(tuning, variant=B.VARIANT_MARCH))):
            assert same_bits(a[1:-1, 1:-1], b[1:-1, 1:-1])


def offset_copy(t, offset):
    """A copy of t whose data starts `offset` elements into a fresh buffer."""
    buf = torch.zeros(t.numel() + offset, dtype=t.dtype, device=t.device)
    view = buf[offset:].view(t.shape)
    view.copy_(t)
    return view


@pytest.mark.parametrize("shapes", [[(12, 9, 32), (7, 20, 50), (30, 5, 80), (3, 4, 64)],
                                    [(12, 9, 33), (7, 20, 51), (5, 5, 64)]],
                         ids=["other-heights", "odd-heights"])
@pytest.mark.parametrize("tuning", [{"chunk": 256, "seg": 4}, {"chunk": 512, "seg": 64}], ids=["c256s4", "c512s64"])
def test_batched_column_heights_outside_the_compiled_set(shapes, tuning):
    """Heights other than 64 / 96 / 128 take the run-time-height path (vector
    loads when nz is even for FP64, element loads when it is odd)."""
    probs = small_problems(shapes, seed=410)
    batch = BT.DeviceBatch(probs, B.F64, DEV)
    plan = batch.plan(tuning)
    batch.advect(plan)
    torch.cuda.synchronize()
    assert plan.error_count() == 0
    for d, p in enumerate(probs):
        ref = oracle.advect_problem(p)
        for g, r in zip(batch.host_outputs(d), ref):
            assert max_rel(g[1:-1, 1:-1], r[1:-1, 1:-1]) <= F64_TOL
        for a, b in zip(batch.fields[d][3:], single_outputs(batch, d, dict(tuning, variant=B.VARIANT_MARCH))):
            assert same_bits(a[1:-1, 1:-1], b[1:-1, 1:-1])


def misaligned_records(batch, d):
    """The batch's records with domain d moved to buffers 8 bytes off a 16-byte boundary."""
    f = [offset_copy(t, 1) for t in batch.fields[d]]
    for o in f[3:]:
        o.fill_(123.0)
    recs = list(batch.records)
    p = batch.problems[d]
    recs[d] = B.domain_record(*f, p.coeffs.tcx, p.coeffs.tcy, *batch.tz[d])
    assert recs[d].u % 16 == 8
    return recs, f


def test_misaligned_record_in_a_vector_plan_is_skipped_and_counted():
    probs = small_problems(SMALL[:4], seed=420)
    batch = BT.DeviceBatch(probs, B.F64, DEV)
    recs, f = misaligned_records(batch, 1)
    plan = batch.plan()
    B.advect_batched(plan, B.domain_args_tensor(recs, DEV))
    torch.cuda.synchronize()
    assert plan.error_count() == 1
    assert all(torch.all(o == 123.0).item() for o in f[3:])
    for d in (0, 2, 3):
        ref = oracle.advect_problem(probs[d])
        for g, r in zip(batch.host_outputs(d), ref):
            assert max_rel(g[1:-1, 1:-1], r[1:-1, 1:-1]) <= F64_TOL


def test_element_aligned_record_in_an_element_plan_is_computed():
    probs = small_problems([(10, 7, 33), (6, 9, 45)], seed=430)
    batch = BT.DeviceBatch(probs, B.F64, DEV)
    recs, f = misaligned_records(batch, 0)
    plan = batch.plan({"chunk": 256, "seg": 4})
    B.advect_batched(plan, B.domain_args_tensor(recs, DEV))
    torch.cuda.synchronize()
    assert plan.error_count() == 0
    ref = oracle.advect_problem(probs[0])
    for g, r in zip(f[3:], ref):
        assert max_rel(g.cpu().numpy()[1:-1, 1:-1], r[1:-1, 1:-1]) <= F64_TOL


def test_shape_mismatch_is_skipped_and_counted():
    probs = small_problems(SMALL[:4], seed=500)
    batch = BT.DeviceBatch(probs, B.F64, DEV)
    bad = list(batch.records)
    rec = B.PwDomainArgs.from_buffer_copy(bytes(bad[2]))
    rec.shape.nx += 1
    bad[2] = rec
    d_bad = B.domain_args_tensor(bad, DEV)
    plan = batch.plan()
    for o in batch.fields[2][3:]:
        o.fill_(123.0)
    B.advect_batched(plan, d_bad)
    torch.cuda.synchronize()
    assert plan.error_count() == 1
    assert all(torch.all(o == 123.0).item() for o in batch.fields[2][3:])
    ref = oracle.advect_problem(probs[1])
    got = batch.host_outputs(1)
    assert max_rel(got[0][1:-1, 1:-1], ref[0][1:-1, 1:-1]) <= F64_TOL


def test_fill_halo_matches_periodic_fill():
    probs = small_problems(seed=600)
    batch = BT.DeviceBatch(probs, B.F64, DEV)
    expect = []
    for d, p in enumerate(probs):
        exp = []
        for f in range(3):
            t = batch.fields[d][f]
            t[0].fill_(-1.0)
            t[-1].fill_(-2.0)
            t[:, 0].fill_(-3.0)
            t[:, -1].fill_(-4.0)
            exp.append(inputs.fill_periodic_halo(t.cpu().numpy().copy()))
        expect.append(exp)
    plan = batch.plan()
    batch.fill_halo(plan)
    torch.cuda.synchronize()
    for d in range(len(probs)):
        for f in range(3):
            assert np.array_equal(batch.fields[d][f].cpu().numpy(), expect[d][f])


def test_perturb_is_deterministic_and_interior_only():
    probs = small_problems(SMALL[:5], seed=700)
    a = BT.DeviceBatch(probs, B.F64, DEV)
    b = BT.DeviceBatch(probs, B.F64, DEV)
    pa, pb = a.plan(), b.plan()
    before = [[t.clone() for t in a.fields[d][:3]] for d in range(len(probs))]
    a.perturb(pa, 42, 1e-3)
    b.perturb(pb, 42, 1e-3)
    torch.cuda.synchronize()
    assert int(a.call.item()) == 1
    for d in range(len(probs)):
        for f in range(3):
            assert same_bits(a.fields[d][f], b.fields[d][f])
        for f in range(2):
            delta = (a.fields[d][f] - before[d][f])
            inner = delta[1:-1, 1:-1]
            assert torch.all(inner.abs() <= 1e-3).item() and torch.any(inner != 0).item()
            assert torch.all(delta[0] == 0).item() and torch.all(delta[:, -1] == 0).item()
        assert same_bits(a.fields[d][2], before[d][2])
    snap = [t.clone() for t in a.fields[0][:2]]
    a.perturb(pa, 42, 1e-3)       # second call: different noise
    torch.cuda.synchronize()
    d2 = a.fields[0][0] - snap[0]
    d1 = snap[0] - before[0][0]
    assert not torch.equal(d1, d2)


M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014), on Python ints."""
    x = (x + 0x9E3779B97F4A7C15) & M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & M64
    return x ^ (x >> 31)


def lowbias32(x):
    """lowbias32 (C. Wellons, 2018) on a numpy uint32 array."""
    x = x ^ (x >> np.uint32(16))
    x = x * np.uint32(0x7FEB352D)
    x = x ^ (x >> np.uint32(15))
    x = x * np.uint32(0x846CA68B)
    return x ^ (x >> np.uint32(16))


def expected_noise(seed, call, dom, nx, ny, nz, q):
    """The documented perturbation r in [-1, 1) of field q (0: u, 1: v) at every
    interior point, shape (nx, ny, nz): key = SplitMix64 of (seed, call,
    domain), then lowbias32(key ^ lowbias32(2 g + q)) with g = k + nz ((j-1) +
    ny (i-1)), its top 24 bits scaled to [0, 2) in FP32, minus 1."""
    k64 = splitmix64(seed ^ splitmix64((call * 0x100000001B3 + dom) & M64))
    key = np.uint32((k64 ^ (k64 >> 32)) & 0xFFFFFFFF)
    g = np.arange(nx * ny * nz, dtype=np.uint32).reshape(nx, ny, nz)
    with np.errstate(over="ignore"):
        h = lowbias32(key ^ lowbias32(np.uint32(2) * g + np.uint32(q)))
    return ((h >> np.uint32(8)).astype(np.float32) * np.float32(2.0 ** -23) - np.float32(1.0)).astype(np.float64)


@pytest.mark.parametrize("tuning", [{"chunk": 256, "seg": 3}, {"chunk": 1024, "seg": 64}, None],
                         ids=["c256s3", "c1024s64", "default"])
def test_perturb_adds_the_documented_noise_at_every_interior_point(tuning):
    """Every interior point of u and v moves by exactly amp * r of the
    counter-based hash, whatever the plan's tiling, on two calls in a row."""
    probs = small_problems(SMALL[:6], seed=710)
    bt = BT.DeviceBatch(probs, B.F64, DEV)
    plan = bt.plan(tuning)
    amp = 1e-3
    for call in range(2):
        before = [[t.cpu().numpy().copy() for t in bt.fields[d][:2]] for d in range(len(probs))]
        bt.perturb(plan, 99, amp)
        torch.cuda.synchronize()
        for d, p in enumerate(probs):
            for q in range(2):
                got = bt.fields[d][q].cpu().numpy()
                want = before[d][q].copy()
                want[1:-1, 1:-1] = before[d][q][1:-1, 1:-1] + amp * expected_noise(99, call, d, p.nx, p.ny, p.nz, q)
                assert np.array_equal(got.view(np.int64), want.view(np.int64)), (tuning, call, d, q)


def test_graph_replays_match_eager_steps():
    probs = small_problems(seed=800)
    ga = BT.DeviceBatch(probs, B.F64, DEV)
    eb = BT.DeviceBatch(probs, B.F64, DEV)
    pa, pb = ga.plan({"chunk": 512, "seg": 16}), eb.plan({"chunk": 512, "seg": 16})
    g = ga.capture_timestep(pa, seed=7, amplitude=1e-3)
    scratch = torch.randn(256, 256, device=DEV)
    for r in range(4):
        g.launch()
        eb.timestep(pb, seed=7, amplitude=1e-3)
        scratch = scratch @ scratch.T / 256.0      # unrelated eager work between replays
        torch.cuda.synchronize()
        assert int(ga.call.item()) == r + 1
        for d in range(len(probs)):
            for x, y in zip(ga.fields[d], eb.fields[d]):
                assert same_bits(x, y), "replay %d domain %d differs from the eager step" % (r, d)
    # the outputs after the last replay are the stencil of the final fields
    for d in (0, 4, len(probs) - 1):
        u, v, w = ga.host_fields(d)
        p = probs[d]
        ref = oracle.advect(u, v, w, p.coeffs.tcx, p.coeffs.tcy, *p.coeffs.arrays())
        for g_, r_ in zip(ga.host_outputs(d), ref):
            assert max_rel(g_[1:-1, 1:-1], r_[1:-1, 1:-1]) <= F64_TOL


def test_autotune_picks_a_valid_candidate():
    probs = small_problems(SMALL[:6], seed=900)
    batch = BT.DeviceBatch(probs, B.F64, DEV)
    cands = [{"variant": 2, "chunk": 256, "seg": 16}, {"variant": 2, "chunk": 512, "seg": 64, "wg_per_cu": 2},
             {"variant": 2, "chunk": 1024, "seg": 8}]
    best, ms, table = BT.autotune(batch, cands, reps=3)
    say("autotune", best, ms, table)
    assert ms > 0 and all(t >= 0 for _, t in table)
    assert any(all(best[k] == c.get(k, 0) for k in ("chunk", "seg")) for c in cands)
    plan = batch.plan(best)
    batch.advect(plan)
    torch.cuda.synchronize()
    for d, p in enumerate(probs):
        ref = oracle.advect_problem(p)
        for g, r in zip(batch.host_outputs(d), ref):
            assert max_rel(g[1:-1, 1:-1], r[1:-1, 1:-1]) <= F64_TOL


def test_autotune_single_domain_default_space():
    p = inputs.make_problem(64, 48, 64, seed=901)
    batch = BT.DeviceBatch([p], B.F64, DEV)
    best, ms, table = BT.autotune(batch, None, reps=2)
    say("single-domain autotune", best, ms, len(table))
    assert ms > 0
    assert sum(1 for _, t in table if t > 0) >= 3


@pytest.mark.parametrize("storage,tuning", [
    (B.F64, None), (B.F64, {"chunk": 512, "seg": 16, "wg_per_cu": 8}),
    (B.F64, {"chunk": 512, "seg": 8, "wg_per_cu": B.WG_ONE_PER_TILE}),
    (B.F32, {"chunk": 512, "seg": 16, "wg_per_cu": B.WG_ONE_PER_TILE})],
    ids=["f64-default", "f64-persistent", "f64-one-per-tile-c512s8", "f32-one-per-tile-c512s16"])
def test_full_384_domain_batch_graph(storage, tuning):
    """The 384-subdomain configuration with the default launch (one workgroup
    per tile), a persistent grid at full occupancy, and the launches the
    autotuner picks on MI355X:
    graph-captured timestep replayed, sampled domains vs the oracle on the
    stored fields (FP64: 1e-12; FP32 storage: FP32 roundoff of the outputs
    plus its compensated arithmetic, 2^-24 + 2e-6)."""
    specs = inputs.batched_specs()
    probs = [inputs.make_domain(s) for s in specs]
    batch = BT.DeviceBatch(probs, storage, DEV)
    tol = F64_TOL if storage == B.F64 else 2.0 ** -24 + 2e-6
    plan = batch.plan(tuning)
    say("384 domains", batch.npoints, plan.info())
    g = batch.capture_timestep(plan, seed=11, amplitude=1e-3)
    for _ in range(3):
        g.launch()
    torch.cuda.synchronize()
    assert plan.error_count() == 0
    for d in (0, 1, 77, 191, 300, 383):
        u, v, w = batch.host_fields(d)
        p = probs[d]
        ref = oracle.advect(u, v, w, p.coeffs.tcx, p.coeffs.tcy, *p.coeffs.arrays())
        for gg, rr in zip(batch.host_outputs(d), ref):
            assert max_rel(gg[1:-1, 1:-1], rr[1:-1, 1:-1]) <= tol
