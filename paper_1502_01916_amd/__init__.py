"""MI355X-native decoding of Group-codec posting lists (Group-Simple,
Group-Scheme, Group-AFOR, Group-PFD; Zhao et al., arXiv 1502.01916).

The compute path lives in ``libgc.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/gc.h``); :mod:`.gc` is its thin ctypes binding.  Importing
this package loads nothing; the binding loads the library on first use and
raises if it is missing.
"""
__all__ = ["gc", "synth"]
