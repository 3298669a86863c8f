"""MI355X-native Piacsek-Williams (PW) momentum advection.

The compute path is the HIP library ``libpwadvect.so`` (C ABI declared in
``include/pw_advect.h``) built from ``csrc/``; ``binding`` wraps it with
ctypes, taking torch device tensors only as memory and streams.  Importing the
package loads nothing: ``binding.lib()`` loads the library on first use and
raises if it has not been built.
"""
__all__ = ["inputs", "metrics", "binding"]


def kernel_sources_sha256() -> str:
    """sha256 over the HIP sources and the C header (identifies a kernel build)."""
    import hashlib
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    files = sorted(os.path.join(here, "csrc", f) for f in os.listdir(os.path.join(here, "csrc"))
                   if f.endswith((".hip", ".hpp", ".h")))
    files.append(os.path.join(os.path.dirname(here), "include", "pw_advect.h"))
    h = hashlib.sha256()
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()
