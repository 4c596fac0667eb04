"""MI355X-native batched simplex cross-map (the hot path of convergent cross
mapping): HIP kernels for gfx950 behind the C ABI in include/ccm.h.

``capi`` is the ctypes binding (same function names as the C ABI);
``synth`` generates seeded synthetic inputs; ``build`` compiles libccm.so.
"""
__all__ = ["capi", "synth", "build"]
