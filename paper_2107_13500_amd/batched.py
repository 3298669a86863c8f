"""Many uneven subdomains in one device pool, driven through the batched C ABI.

``DeviceBatch`` lays every domain's six field arrays out in one device
allocation (each array 256-byte aligned), keeps the per-level coefficients in
a second pool, and holds the device array of ``pw_domain_args`` records that
``pw_advect_batched``, ``pw_fill_halo_batched`` and ``pw_perturb_batched``
read.  ``capture_timestep`` records one timestep -- perturb u and v, refill
the periodic halos, compute su, sv, sw of every domain -- into a HIP graph
through the library's graph entry points, then replayed once per call.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import binding as B
from . import inputs

ALIGN = 256


def _round_up(x: int, a: int) -> int:
    return (x + a - 1) // a * a


class DeviceBatch:
    def __init__(self, problems: Sequence[inputs.Problem], storage: int, device, scales: Optional[list] = None):
        import torch
        self.problems = list(problems)
        self.storage = storage
        self.device = torch.device(device)
        dt = B.torch_dtype(storage)
        esize = torch.tensor([], dtype=dt).element_size()
        # field pool layout
        offs = []
        total = 0
        for p in self.problems:
            n = (p.nx + 2) * (p.ny + 2) * p.nz
            o = []
            for _ in range(6):
                o.append(total)
                total = _round_up(total + n * esize, ALIGN)
            offs.append(o)
        self.pool = torch.zeros(total, dtype=torch.uint8, device=self.device)
        coef = np.concatenate([np.concatenate(p.coeffs.arrays()) for p in self.problems])
        self.coef_pool = torch.from_numpy(coef).to(self.device)
        self.fields: List[list] = []     # per domain: [u, v, w, su, sv, sw] tensors of shape (nx+2, ny+2, nz)
        self.tz: List[list] = []
        self.scales = []
        ci = 0
        for d, p in enumerate(self.problems):
            n = (p.nx + 2) * (p.ny + 2) * p.nz
            views = [self.pool[o:o + n * esize].view(dt).view(p.nx + 2, p.ny + 2, p.nz) for o in offs[d]]
            if scales is not None:
                sc = scales[d]
            else:
                sc = B.make_scales(*inputs.storage_scales(p, B.DTYPE_NAMES[storage]))
            for f, a in enumerate((p.u, p.v, p.w)):
                views[f].copy_(B.to_storage(a, storage, float(sc.in_scale[f]), self.device))
            tz = [self.coef_pool[ci + q * p.nz: ci + (q + 1) * p.nz] for q in range(4)]
            ci += 4 * p.nz
            self.fields.append(views)
            self.tz.append(tz)
            self.scales.append(sc)
        self.records = [B.domain_record(*f, p.coeffs.tcx, p.coeffs.tcy, *tz, scales=sc)
                        for f, p, tz, sc in zip(self.fields, self.problems, self.tz, self.scales)]
        self.d_args = B.domain_args_tensor(self.records, self.device)
        self.call = torch.zeros(1, dtype=torch.int64, device=self.device)

    @property
    def shapes(self):
        return [r.shape for r in self.records]

    @property
    def npoints(self) -> int:
        return sum(p.npoints for p in self.problems)

    def plan(self, tuning=None) -> B.Plan:
        return B.Plan(self.storage, self.shapes, tuning)

    def advect(self, plan: B.Plan, stream=None):
        B.advect_batched(plan, self.d_args, stream)

    def fill_halo(self, plan: B.Plan, stream=None):
        B.fill_halo_batched(plan, self.d_args, stream)

    def perturb(self, plan: B.Plan, seed: int, amplitude: float, stream=None):
        B.perturb_batched(plan, self.d_args, seed, self.call, amplitude, stream)

    def timestep(self, plan: B.Plan, seed: int, amplitude: float, stream=None):
        """One repeated-call step: perturb u, v; refill halos; su, sv, sw of every domain."""
        self.perturb(plan, seed, amplitude, stream)
        self.fill_halo(plan, stream)
        self.advect(plan, stream)

    def capture_timestep(self, plan: B.Plan, seed: int, amplitude: float, nsteps: int = 1) -> B.Graph:
        """Record `nsteps` timesteps into a HIP graph (pw_graph_capture_timestep);
        ``launch(stream)`` replays them."""
        return B.Graph.timestep(plan, self.d_args, seed, self.call, amplitude, nsteps)

    def per_domain_plans(self, tuning=None) -> List[B.Plan]:
        return [B.Plan(self.storage, [r.shape], tuning) for r in self.records]

    def advect_per_domain(self, plans: Sequence[B.Plan], stream=None):
        """The same work as ``advect`` as one pw_advect launch per domain."""
        for f, tz, p, sc, pl in zip(self.fields, self.tz, self.problems, self.scales, plans):
            B.advect(pl, *f, p.coeffs.tcx, p.coeffs.tcy, *tz,
                     scales=sc if self.storage in B.SCALED else None, stream=stream)

    def host_fields(self, d: int):
        """u, v, w of domain d copied back as float64 numpy arrays (descaled)."""
        return [B.from_storage(self.fields[d][f], self.storage, float(self.scales[d].in_scale[f]))
                for f in range(3)]

    def host_outputs(self, d: int):
        return [B.from_storage(self.fields[d][3 + f], self.storage, float(self.scales[d].out_scale[f]))
                for f in range(3)]


def autotune(batch: DeviceBatch, candidates: Optional[Sequence[dict]] = None, reps: int = 5):
    """Run the library's autotuner on a batch; returns (best tuning dict, best ms, [(tuning, ms)])."""
    import ctypes
    l = B.lib()
    shapes = (B.PwShape * len(batch.records))(*batch.shapes)
    if candidates is None:
        n = l.pw_autotune_candidates(1 if len(batch.records) > 1 else 0, None, 0)
        arr = (B.PwTuning * n)()
        l.pw_autotune_candidates(1 if len(batch.records) > 1 else 0, arr, n)
    else:
        n = len(candidates)
        arr = (B.PwTuning * n)(*[B.make_tuning(c) for c in candidates])
    best = B.PwTuning()
    best_ms = ctypes.c_float(0)
    all_ms = (ctypes.c_float * n)()
    h = (B.PwDomainArgs * len(batch.records))(*batch.records)
    B.check(l.pw_autotune(batch.storage, shapes, len(batch.records), ctypes.cast(h, ctypes.c_void_p),
                          batch.d_args.data_ptr(), arr, n, reps, ctypes.byref(best), ctypes.byref(best_ms),
                          all_ms), "pw_autotune")
    as_dict = lambda t: {f: getattr(t, f) for f, _ in B.PwTuning._fields_}
    return as_dict(best), float(best_ms.value), [(as_dict(arr[i]), float(all_ms[i])) for i in range(n)]
