"""ctypes binding of ``libpwadvect.so`` (C ABI: ``include/pw_advect.h``).

Argument marshalling only: torch tensors supply device pointers and
``torch.cuda`` streams supply hipStream_t handles; every step of the stencil
runs in the library's HIP kernels.  The library is loaded on first use and
there is no fallback: if it has not been built, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_uint64, c_ulonglong, c_void_p
from typing import List, Optional, Sequence

LIBRARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpwadvect.so")

PW_OK = 0
STATUS_NAMES = {
    0: "PW_OK", -1: "PW_ERR_INVALID_ARG", -2: "PW_ERR_UNSUPPORTED", -3: "PW_ERR_ALIAS",
    -4: "PW_ERR_ALIGNMENT", -5: "PW_ERR_OUT_OF_MEMORY", -6: "PW_ERR_HIP", -7: "PW_ERR_CAPTURE",
    -8: "PW_ERR_PLAN_MISMATCH",
}
F64, F32, BF16, F16, I16, I32 = 0, 1, 2, 3, 4, 5
SCALED = (BF16, F16, I16, I32)
FIXED_RANGE = {I16: (-32768, 32767), I32: (-2147483648, 2147483647)}
VARIANT_AUTO, VARIANT_DIRECT, VARIANT_MARCH = 0, 1, 2
WG_ONE_PER_TILE = -1   # pw_tuning.wg_per_cu: one workgroup per tile instead of a persistent grid
DTYPE_NAMES = {F64: "f64", F32: "f32", BF16: "bf16", F16: "f16", I16: "i16", I32: "i32"}


class PwShape(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("reserved", c_int32),
                ("sy", c_int64), ("sx", c_int64)]


class PwTuning(ctypes.Structure):
    _fields_ = [("variant", c_int32), ("chunk", c_int32), ("seg", c_int32), ("block", c_int32),
                ("wg_per_cu", c_int32)]


class PwScales(ctypes.Structure):
    _fields_ = [("in_scale", c_float * 3), ("out_scale", c_float * 3)]


class PwPlanInfo(ctypes.Structure):
    _fields_ = [("storage", c_int32), ("ndomains", c_int32), ("variant", c_int32), ("chunk", c_int32),
                ("seg", c_int32), ("block", c_int32), ("workgroups", c_int64), ("tiles", c_int64),
                ("lds_bytes", c_int64), ("points", c_int64), ("batched_workgroups", c_int64)]


class PwDomainArgs(ctypes.Structure):
    _fields_ = [("shape", PwShape),
                ("u", c_void_p), ("v", c_void_p), ("w", c_void_p),
                ("su", c_void_p), ("sv", c_void_p), ("sw", c_void_p),
                ("tcx", c_double), ("tcy", c_double),
                ("tzc1", c_void_p), ("tzc2", c_void_p), ("tzd1", c_void_p), ("tzd2", c_void_p),
                ("scales", PwScales)]


#: every function the header declares, with (restype, argtypes)
SIGNATURES = {
    "pw_advect_plan": (c_int32, [POINTER(c_void_p), c_int32, POINTER(PwShape), c_int32, POINTER(PwTuning)]),
    "pw_plan_destroy": (c_int32, [c_void_p]),
    "pw_plan_get_info": (c_int32, [c_void_p, POINTER(PwPlanInfo)]),
    "pw_advect": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                            POINTER(PwScales), c_void_p]),
    "pw_advect_batched": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "pw_advect_batched_noalloc": (c_int32, [c_int32, POINTER(PwShape), c_int32, c_void_p, POINTER(PwTuning),
                                            c_void_p, c_void_p]),
    "pw_fill_halo_batched": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "pw_perturb_batched": (c_int32, [c_void_p, c_int32, c_void_p, c_uint64, c_void_p, c_double, c_void_p]),
    "pw_plan_error_count": (c_int32, [c_void_p, POINTER(c_ulonglong)]),
    "pw_graph_begin": (c_int32, [POINTER(c_void_p)]),
    "pw_graph_end": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "pw_graph_capture_timestep": (c_int32, [c_void_p, c_int32, c_void_p, c_uint64, c_void_p, c_double, c_int32,
                                            POINTER(c_void_p)]),
    "pw_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "pw_graph_destroy": (c_int32, [c_void_p]),
    "pw_autotune": (c_int32, [c_int32, POINTER(PwShape), c_int32, c_void_p, c_void_p, POINTER(PwTuning),
                              c_int32, c_int32, POINTER(PwTuning), POINTER(c_float), POINTER(c_float)]),
    "pw_autotune_candidates": (c_int32, [c_int32, POINTER(PwTuning), c_int32]),
    "pw_stream_plan_create": (c_int32, [POINTER(c_void_p), c_int32, POINTER(PwShape), c_int32, c_int32, c_int32,
                                        POINTER(PwTuning)]),
    "pw_stream_plan_destroy": (c_int32, [c_void_p]),
    "pw_advect_host": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(PwScales)]),
    "pw_probe_copy": (c_int32, [POINTER(c_void_p), POINTER(c_void_p), c_int32, c_int64, c_int32, c_void_p]),
    "pw_probe_bandwidth": (c_int32, [POINTER(c_void_p), c_int32, POINTER(c_void_p), c_int32, c_int64, c_int32,
                                     c_int32, c_void_p, c_void_p]),
    "pw_probe_march": (c_int32, [c_void_p] * 6 + [POINTER(PwShape), c_int32, c_void_p]),
    "pw_status_string": (ctypes.c_char_p, [c_int32]),
    "pw_last_hip_error": (c_int32, []),
}

_lib = None


class PwError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        hip = _lib.pw_last_hip_error() if (_lib is not None and status == -6) else 0
        self.hip_error = hip
        msg = "%s failed: %s (%s)" % (where, STATUS_NAMES.get(status, status),
                                      _lib.pw_status_string(status).decode() if _lib else "?")
        if hip:
            msg += ", hipError %d" % hip
        super().__init__(msg)


def lib(path: Optional[str] = None):
    """Load the HIP library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIBRARY
    if not os.path.exists(p):
        raise FileNotFoundError(
            "HIP library %s is not built; run `python -m paper_2107_13500_amd.build` "
            "(or __graft_entry__.build())" % p)
    l = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(l, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = l
    return l


def check(status: int, where: str):
    if status != PW_OK:
        raise PwError(status, where)


# ----------------------------------------------------------------------------
# torch plumbing (memory and streams only)
# ----------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def storage_of(dtype) -> int:
    torch = _torch()
    table = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16, torch.int16: I16,
             torch.int32: I32}
    if dtype not in table:
        raise TypeError("unsupported field dtype %s" % dtype)
    return table[dtype]


def torch_dtype(storage: int):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16,
            I16: torch.int16, I32: torch.int32}[storage]


def to_storage(a, storage: int, scale: float = 1.0, device=None):
    """Host float64 numpy array -> tensor of the storage type (scaled; fixed
    point rounded to nearest even and saturated), optionally moved to `device`."""
    torch = _torch()
    t = torch.from_numpy(a)
    if device is not None:
        t = t.to(device)
    if storage in SCALED and scale != 1.0:
        t = t * scale
    if storage in FIXED_RANGE:
        t = torch.round(t).clamp_(*FIXED_RANGE[storage])
    return t.to(torch_dtype(storage))


def from_storage(t, storage: int, scale: float = 1.0):
    """Device/host tensor of a storage type -> float64 numpy array (descaled)."""
    a = t.double().cpu().numpy()
    return a / scale if (storage in SCALED and scale != 1.0) else a


def stream_handle(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def shape_of(t) -> PwShape:
    """pw_shape of a halo'd field tensor (nx+2, ny+2, nz) with a unit k stride."""
    if t.dim() != 3 or t.stride(2) != 1:
        raise ValueError("fields must be (nx+2, ny+2, nz) tensors with a contiguous k axis")
    return PwShape(t.shape[0] - 2, t.shape[1] - 2, t.shape[2], 0, t.stride(1), t.stride(0))


def make_tuning(tuning=None) -> Optional[PwTuning]:
    if tuning is None:
        return None
    if isinstance(tuning, PwTuning):
        return tuning
    return PwTuning(int(tuning.get("variant", 0)), int(tuning.get("chunk", 0)), int(tuning.get("seg", 0)),
                    int(tuning.get("block", 0)), int(tuning.get("wg_per_cu", 0)))


def make_scales(in_scale=(1.0, 1.0, 1.0), out_scale=(1.0, 1.0, 1.0)) -> PwScales:
    s = PwScales()
    for f in range(3):
        s.in_scale[f] = float(in_scale[f])
        s.out_scale[f] = float(out_scale[f])
    return s


class Plan:
    """Owning wrapper of a pw_plan."""

    def __init__(self, storage: int, shapes: Sequence[PwShape], tuning=None):
        l = lib()
        arr = (PwShape * len(shapes))(*shapes)
        h = c_void_p()
        t = make_tuning(tuning)
        check(l.pw_advect_plan(ctypes.byref(h), int(storage), arr, len(shapes),
                               ctypes.byref(t) if t is not None else None), "pw_advect_plan")
        self.handle = h
        self.storage = storage
        self.ndomains = len(shapes)
        self.shapes = list(shapes)

    def info(self) -> dict:
        i = PwPlanInfo()
        check(lib().pw_plan_get_info(self.handle, ctypes.byref(i)), "pw_plan_get_info")
        return {f: getattr(i, f) for f, _ in PwPlanInfo._fields_}

    def error_count(self) -> int:
        n = c_ulonglong(0)
        check(lib().pw_plan_error_count(self.handle, ctypes.byref(n)), "pw_plan_error_count")
        return int(n.value)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(lib().pw_plan_destroy(self.handle), "pw_plan_destroy")
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _normalised(s: PwShape):
    sy = s.sy or s.nz
    return (s.nx, s.ny, s.nz, sy, s.sx or (s.ny + 2) * sy)


def check_fields(storage: int, shape: PwShape, fields, tz) -> None:
    """Raise ValueError unless the six field tensors are CUDA tensors of the
    storage dtype, on one device, each spanning `shape` (extents and strides),
    and the four coefficient tensors are contiguous CUDA float64 tensors of at
    least nz values on the same device.  Run before any pointer reaches the
    library, whose kernels trust these extents."""
    torch = _torch()
    want = _normalised(shape)
    dt = torch_dtype(storage)
    dev = fields[0].device if len(fields) else None
    for name, t in zip(("u", "v", "w", "su", "sv", "sw"), fields):
        if t.dtype != dt:
            raise ValueError("%s has dtype %s; the plan stores %s" % (name, t.dtype, dt))
        if _normalised(shape_of(t)) != want:
            raise ValueError("%s has shape %s and strides %s; the plan expects (nx, ny, nz, sy, sx) = %s"
                             % (name, tuple(t.shape), t.stride(), want))
    for name, t in zip(("tzc1", "tzc2", "tzd1", "tzd2"), tz):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < shape.nz:
            raise ValueError("%s must be a contiguous float64 tensor of at least nz = %d values" % (name, shape.nz))
    for name, t in zip(("u", "v", "w", "su", "sv", "sw", "tzc1", "tzc2", "tzd1", "tzd2"), (*fields, *tz)):
        if not t.is_cuda or t.device != dev:
            raise ValueError("%s must be a CUDA tensor on %s" % (name, dev))


def advect(plan: Plan, u, v, w, su, sv, sw, tcx: float, tcy: float, tzc1, tzc2, tzd1, tzd2,
           scales: Optional[PwScales] = None, stream=None) -> None:
    """pw_advect on torch device tensors (asynchronous on `stream`)."""
    if plan.ndomains != 1:
        raise ValueError("pw_advect needs a single-domain plan")
    check_fields(plan.storage, plan.shapes[0], (u, v, w, su, sv, sw), (tzc1, tzc2, tzd1, tzd2))
    st = lib().pw_advect(plan.handle, u.data_ptr(), v.data_ptr(), w.data_ptr(),
                         su.data_ptr(), sv.data_ptr(), sw.data_ptr(), float(tcx), float(tcy),
                         tzc1.data_ptr(), tzc2.data_ptr(), tzd1.data_ptr(), tzd2.data_ptr(),
                         ctypes.byref(scales) if scales is not None else None, stream_handle(stream))
    check(st, "pw_advect")


def advect_batched(plan: Plan, d_args, stream=None) -> None:
    """pw_advect_batched; ``d_args`` is a uint8 device tensor holding the pw_domain_args array."""
    check(lib().pw_advect_batched(plan.handle, plan.ndomains, d_args.data_ptr(), stream_handle(stream)),
          "pw_advect_batched")


def advect_batched_noalloc(storage: int, shapes: Sequence[PwShape], d_args, tuning=None, d_skipped=None,
                           stream=None) -> None:
    """pw_advect_batched_noalloc: the batched call without a plan (nothing is
    allocated); ``d_skipped`` is an optional int64 device tensor of one element."""
    arr = (PwShape * len(shapes))(*shapes)
    t = make_tuning(tuning)
    check(lib().pw_advect_batched_noalloc(int(storage), arr, len(shapes), d_args.data_ptr(),
                                          ctypes.byref(t) if t is not None else None,
                                          d_skipped.data_ptr() if d_skipped is not None else None,
                                          stream_handle(stream)), "pw_advect_batched_noalloc")


def fill_halo_batched(plan: Plan, d_args, stream=None) -> None:
    check(lib().pw_fill_halo_batched(plan.handle, plan.ndomains, d_args.data_ptr(), stream_handle(stream)),
          "pw_fill_halo_batched")


def perturb_batched(plan: Plan, d_args, seed: int, d_call, amplitude: float, stream=None) -> None:
    check(lib().pw_perturb_batched(plan.handle, plan.ndomains, d_args.data_ptr(), int(seed),
                                   d_call.data_ptr(), float(amplitude), stream_handle(stream)),
          "pw_perturb_batched")


class RawStream:
    """A hipStream_t handle the library owns (a recording stream), usable
    wherever the binding takes a torch stream."""

    def __init__(self, handle: int):
        self.cuda_stream = handle


class Graph:
    """Owning wrapper of a pw_graph (an instantiated HIP graph of library calls)."""

    def __init__(self, handle: c_void_p):
        self.handle = handle

    @classmethod
    def timestep(cls, plan: Plan, d_args, seed: int, d_call, amplitude: float, nsteps: int = 1) -> "Graph":
        """pw_graph_capture_timestep: `nsteps` perturb + halo + advect steps of a batched plan."""
        h = c_void_p()
        check(lib().pw_graph_capture_timestep(plan.handle, plan.ndomains, d_args.data_ptr(), int(seed),
                                              d_call.data_ptr(), float(amplitude), int(nsteps), ctypes.byref(h)),
              "pw_graph_capture_timestep")
        return cls(h)

    @classmethod
    def record(cls, fn) -> "Graph":
        """Record the library calls ``fn(stream)`` issues on the recording
        stream it is given (pw_graph_begin / pw_graph_end; the stream belongs
        to the recording and is destroyed with it)."""
        h = c_void_p()
        check(lib().pw_graph_begin(ctypes.byref(h)), "pw_graph_begin")
        rs = RawStream(h.value)
        g = c_void_p()
        try:
            fn(rs)
        except BaseException:
            lib().pw_graph_end(h, ctypes.byref(g))   # abandon the recording (frees its stream)
            if g.value:
                lib().pw_graph_destroy(g)
            raise
        check(lib().pw_graph_end(h, ctypes.byref(g)), "pw_graph_end")
        return cls(g)

    def launch(self, stream=None) -> None:
        check(lib().pw_graph_launch(self.handle, stream_handle(stream)), "pw_graph_launch")

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(lib().pw_graph_destroy(self.handle), "pw_graph_destroy")
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_copy(srcs, dsts, nbytes: int, workgroups: int = 0, stream=None) -> None:
    """pw_probe_copy over lists of device tensors (HBM calibration)."""
    n = len(srcs)
    sp = (c_void_p * n)(*[t.data_ptr() for t in srcs])
    dp = (c_void_p * n)(*[t.data_ptr() for t in dsts])
    check(lib().pw_probe_copy(sp, dp, n, int(nbytes), int(workgroups), stream_handle(stream)), "pw_probe_copy")


PROBE_NT_LOADS, PROBE_CACHED_STORES, PROBE_UNROLL4 = 1, 2, 4


def probe_bandwidth(srcs, dsts, nbytes: int, workgroups: int = 0, flags: int = 0, sink=None, stream=None) -> None:
    """pw_probe_bandwidth: read ``srcs`` and write ``dsts`` (lists of device
    tensors, either may be empty); ``sink`` is a device tensor of at least 16
    bytes per workgroup, needed when ``dsts`` is empty."""
    sp = (c_void_p * max(1, len(srcs)))(*[t.data_ptr() for t in srcs])
    dp = (c_void_p * max(1, len(dsts)))(*[t.data_ptr() for t in dsts])
    check(lib().pw_probe_bandwidth(sp, len(srcs), dp, len(dsts), int(nbytes), int(workgroups), int(flags),
                                   sink.data_ptr() if sink is not None else None, stream_handle(stream)),
          "pw_probe_bandwidth")


def probe_march(fields, seg: int, stream=None) -> None:
    """pw_probe_march on six FP64 device tensors (u, v, w, su, sv, sw) of one
    domain: the march kernel's access pattern without LDS or arithmetic; the
    interior columns of su, sv, sw are overwritten."""
    if len(fields) != 6:
        raise ValueError("probe_march needs the six arrays u, v, w, su, sv, sw")
    shape = shape_of(fields[0])
    check_fields(F64, shape, fields, ())
    check(lib().pw_probe_march(*[t.data_ptr() for t in fields], ctypes.byref(shape), int(seg),
                               stream_handle(stream)), "pw_probe_march")


class StreamPlan:
    """Owning wrapper of a pw_stream_plan (host-resident domain)."""

    def __init__(self, storage: int, shape: PwShape, chunk: int = 64, nbuffers: int = 3, bulk: bool = False,
                 tuning=None):
        h = c_void_p()
        t = make_tuning(tuning)
        check(lib().pw_stream_plan_create(ctypes.byref(h), int(storage), ctypes.byref(shape), int(chunk),
                                          int(nbuffers), 1 if bulk else 0,
                                          ctypes.byref(t) if t is not None else None), "pw_stream_plan_create")
        self.handle = h
        self.storage = storage

    def run(self, u, v, w, su, sv, sw, tcx, tcy, tzc1, tzc2, tzd1, tzd2, scales: Optional[PwScales] = None):
        """pw_advect_host on host tensors (blocking)."""
        check(lib().pw_advect_host(self.handle, u.data_ptr(), v.data_ptr(), w.data_ptr(), su.data_ptr(),
                                   sv.data_ptr(), sw.data_ptr(), float(tcx), float(tcy), tzc1.data_ptr(),
                                   tzc2.data_ptr(), tzd1.data_ptr(), tzd2.data_ptr(),
                                   ctypes.byref(scales) if scales is not None else None), "pw_advect_host")

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(lib().pw_stream_plan_destroy(self.handle), "pw_stream_plan_destroy")
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def domain_args_tensor(records: Sequence[PwDomainArgs], device):
    """Copy an array of pw_domain_args to a device uint8 tensor (synchronous)."""
    torch = _torch()
    arr = (PwDomainArgs * len(records))(*records)
    raw = bytes(memoryview(arr).cast("B"))
    host = torch.frombuffer(bytearray(raw), dtype=torch.uint8)
    return host.to(device)


def domain_record(u, v, w, su, sv, sw, tcx, tcy, tzc1, tzc2, tzd1, tzd2,
                  scales: Optional[PwScales] = None) -> PwDomainArgs:
    """pw_domain_args of one domain's device tensors (checked like ``advect``'s)."""
    r = PwDomainArgs()
    r.shape = shape_of(u)
    check_fields(storage_of(u.dtype), r.shape, (u, v, w, su, sv, sw), (tzc1, tzc2, tzd1, tzd2))
    r.u, r.v, r.w = u.data_ptr(), v.data_ptr(), w.data_ptr()
    r.su, r.sv, r.sw = su.data_ptr(), sv.data_ptr(), sw.data_ptr()
    r.tcx, r.tcy = float(tcx), float(tcy)
    r.tzc1, r.tzc2, r.tzd1, r.tzd2 = tzc1.data_ptr(), tzc2.data_ptr(), tzd1.data_ptr(), tzd2.data_ptr()
    r.scales = scales if scales is not None else make_scales()
    return r


# ----------------------------------------------------------------------------
# convenience: one domain, fields already on the device
# ----------------------------------------------------------------------------
def pooled_fields(shape, dtype, device, count: int = 6, align_bytes: int = 256):
    """`count` arrays of `shape` as views into ONE allocation, back to back
    (each start rounded up to `align_bytes`).  The recommended HBM layout for
    a domain's u, v, w, su, sv, sw: separately allocated arrays share the
    allocator's large alignment, so equal offsets in the six streams can land
    on the same HBM channels; on MI355X that made the 2048 x 2048 x 64 FP64
    call 5% slower on some placements, while packed arrays ran at the fast
    rate on every placement tried."""
    torch = _torch()
    n = 1
    for e in shape:
        n *= int(e)
    esize = torch.empty((), dtype=dtype).element_size()
    step = -(-n * esize // align_bytes) * align_bytes // esize
    buf = torch.empty(count * step, dtype=dtype, device=device)
    return [buf[k * step:k * step + n].view(*shape) for k in range(count)]


class DeviceDomain:
    """Device copies of one domain's fields and coefficients plus output buffers.

    ``u, v, w`` are (nx+2, ny+2, nz) tensors of the storage dtype; the four
    coefficient arrays stay float64 (the ABI keeps them FP64 for every
    storage type).  ``outputs`` (optional) are caller-provided su, sv, sw
    buffers, e.g. from ``pooled_fields``; otherwise new tensors.  Outputs
    start zeroed so their (never written) halos are 0.
    """

    def __init__(self, u, v, w, tcx, tcy, tzc1, tzc2, tzd1, tzd2, scales: Optional[PwScales] = None,
                 outputs=None):
        torch = _torch()
        self.u, self.v, self.w = u, v, w
        if outputs is None:
            self.su, self.sv, self.sw = (torch.zeros_like(u) for _ in range(3))
        else:
            self.su, self.sv, self.sw = outputs
            for o in outputs:
                if o.shape != u.shape or o.dtype != u.dtype or o.device != u.device:
                    raise ValueError("outputs must match u in shape, dtype and device")
                o.zero_()
        self.tcx, self.tcy = float(tcx), float(tcy)
        self.tz = [t.to(device=u.device, dtype=torch.float64).contiguous() for t in (tzc1, tzc2, tzd1, tzd2)]
        self.scales = scales

    @property
    def outputs(self):
        return self.su, self.sv, self.sw

    def record(self) -> PwDomainArgs:
        return domain_record(self.u, self.v, self.w, self.su, self.sv, self.sw, self.tcx, self.tcy,
                             *self.tz, scales=self.scales)

    def run(self, plan: Plan, stream=None):
        advect(plan, self.u, self.v, self.w, self.su, self.sv, self.sw, self.tcx, self.tcy, *self.tz,
               scales=self.scales, stream=stream)
