"""MI355X-native Piacsek-Williams (PW) momentum advection.

The compute path is the HIP library ``libpwadvect.so`` (C ABI declared in
``include/pw_advect.h``) built from ``csrc/``; ``binding`` wraps it with
ctypes, taking torch device tensors only as memory and streams.  Importing the
package loads nothing: ``binding.lib()`` loads the library on first use and
raises if it has not been built.
"""
__all__ = ["inputs", "metrics", "binding"]


#: sources the single-domain kernels are compiled from
KERNEL_SOURCES = ("pw_types.hpp", "pw_stencil.hpp", "pw_kernels.hpp", "pw_plan.hpp", "pw_advect.hip")


def kernel_sources_sha256() -> str:
    """sha256 over the sources of the single-domain kernels (identifies a kernel build)."""
    import hashlib
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(here, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()
