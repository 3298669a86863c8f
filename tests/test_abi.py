"""The C ABI without a GPU: declared symbols are exported, struct layouts match.

No compute call is made here; the library is only loaded (loading the HIP
runtime needs no device).
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2107_13500_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pw_advect.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(pw_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("pw_advect_plan", "pw_advect", "pw_advect_batched", "pw_plan_destroy",
                     "pw_status_string", "pw_last_hip_error"):
        assert required in names


def test_binding_covers_every_declared_function():
    assert sorted(B.SIGNATURES) == declared_functions()


def test_library_exports_every_declared_symbol():
    if not os.path.exists(B.LIBRARY):
        pytest.fail("libpwadvect.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(B.LIBRARY)
    for name in declared_functions():
        assert hasattr(lib, name), "missing export %s" % name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIBRARY], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pw_\w+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_status_strings_without_a_device():
    lib = B.lib()
    for code in B.STATUS_NAMES:
        assert lib.pw_status_string(code)
    assert lib.pw_last_hip_error() == 0


def test_plan_rejects_out_of_range_shapes_without_a_device():
    """Shape checks run on the host before any device call: strides or
    extents whose offsets would overflow, and 32-bit index limits."""
    lib = B.lib()
    big = 1 << 62
    bad = [B.PwShape(4, 4, 8, 0, big, 0),                 # sy: (ny + 2) sy would overflow
           B.PwShape(4, 4, 8, 0, 0, big),                 # sx: offsets beyond 2^48 elements
           B.PwShape(4, 2 ** 31 - 1, 8, 0, 0, 0),         # ny + 2 overflows 32 bits
           B.PwShape(2 ** 31 - 1, 4, 8, 0, 0, 0),         # plane index nx + 1 beyond 32 bits
           B.PwShape(4, 2 ** 26, 64, 0, 0, 0),            # (ny + 2) nz >= 2^31
           B.PwShape(4, 4, 8, 0, -8, 0), B.PwShape(4, 4, 8, 0, 0, -1)]
    for s in bad:
        h = ctypes.c_void_p()
        assert lib.pw_advect_plan(ctypes.byref(h), B.F64, (B.PwShape * 1)(s), 1, None) == -1, \
            (s.nx, s.ny, s.nz, s.sy, s.sx)
        assert not h.value


PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "pw_advect.h"
#define P(T, F) printf(#T " " #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("pw_shape sizeof %zu\n", sizeof(pw_shape));
  printf("pw_tuning sizeof %zu\n", sizeof(pw_tuning));
  printf("pw_scales sizeof %zu\n", sizeof(pw_scales));
  printf("pw_plan_info sizeof %zu\n", sizeof(pw_plan_info));
  printf("pw_domain_args sizeof %zu\n", sizeof(pw_domain_args));
  P(pw_shape, sy); P(pw_shape, sx);
  P(pw_domain_args, u); P(pw_domain_args, tcx); P(pw_domain_args, tzc1); P(pw_domain_args, scales);
  P(pw_plan_info, workgroups); P(pw_plan_info, batched_workgroups);
  return 0;
}
"""


def test_ctypes_layouts_match_the_header(tmp_path):
    src = tmp_path / "probe.c"
    exe = tmp_path / "probe"
    src.write_text(PROBE)
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in lines:
        if ln.strip():
            t, f, n = ln.split()
            got[(t, f)] = int(n)
    cls = {"pw_shape": B.PwShape, "pw_tuning": B.PwTuning, "pw_scales": B.PwScales,
           "pw_plan_info": B.PwPlanInfo, "pw_domain_args": B.PwDomainArgs}
    for (t, f), n in got.items():
        if f == "sizeof":
            assert ctypes.sizeof(cls[t]) == n, t
        else:
            assert getattr(cls[t], f).offset == n, (t, f)
