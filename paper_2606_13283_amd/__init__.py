"""MI355X-native FP64 orbital-free SCF hot path (Archê method).

The compute path lives in ``libarche.so`` (hand-written HIP for gfx950 behind
the C ABI declared in ``include/arche.h``); ``arche`` is its thin ctypes
binding.  Importing this package loads nothing; ``arche.load()`` does, and
fails loudly when the library is missing.
"""
