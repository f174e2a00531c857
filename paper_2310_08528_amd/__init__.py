"""MI355X-native deform-then-splat render of 4D Gaussian Splatting.

The compute path is the HIP library ``libg4d.so`` (built from ``csrc/``)
behind a C ABI declared in ``include/g4d.h``; ``g4d`` is its thin ctypes
binding and ``synth`` holds the seeded synthetic inputs.  Nothing is loaded
at import time.
"""
__all__ = ["g4d", "synth"]
