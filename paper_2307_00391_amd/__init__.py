"""MI355X-native state-vector simulator for gate-level HHL (QLSA-1).

The compute path is the HIP library ``libsv.so`` built from ``csrc/`` for
gfx950 and reached through the C ABI declared in ``include/sv.h``;
``binding`` is a thin ctypes layer over it.  Importing the package does not
load the library: ``binding.lib()`` does, and raises if it is missing.
"""
__all__ = ["binding", "inputs", "metrics"]
