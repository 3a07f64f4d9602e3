"""MI355X-native sensor-prior featuremetric LM pose solver (PiLoT v2 hot path).

The solver lives in libpilot.so (hand-written HIP for gfx950, C ABI in
include/pilot.h); `pilot` is its argument-marshalling binding and `build`
compiles it in-tree.  Importing this package loads nothing.
"""
__all__ = ["build", "pilot"]
