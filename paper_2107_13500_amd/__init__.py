"""MI355X-native Piacsek-Williams (PW) momentum advection.

The compute path is the HIP library ``libpwadvect.so`` (C ABI declared in
``include/pw_advect.h``) built from ``csrc/``; ``binding`` wraps it with
ctypes, taking torch device tensors only as memory and streams.  Importing the
package loads nothing: ``binding.lib()`` loads the library on first use and
raises if it has not been built.
"""
__all__ = ["inputs", "metrics", "binding"]
