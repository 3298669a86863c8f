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


def _strip_comments(text: str) -> str:
    """C/C++ source without comments and with whitespace runs collapsed."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                       # string or character literal
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_sources_sha256() -> str:
    """sha256 identifying a build of the single-domain kernels: their sources
    with comments and layout removed, and the compiler flags."""
    import hashlib
    import os
    from . import build
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    # flags that shape the code (include paths left out: they are machine-specific)
    h.update(" ".join(f for f in build.HIPCC_FLAGS if f.startswith("-") and f != "-I").encode())
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(here, name), encoding="utf-8") as f:
            h.update(_strip_comments(f.read()).encode())
    return h.hexdigest()
