"""MI355X (gfx950) Oriented FAST over an image pyramid.

The detector is the C-ABI library libof_hip.so (include/of.h); ``ofhip`` is its thin
Python binding, ``tune`` the autotuner of the batched call's launch shape, ``serve`` the
continuous-batching request loop and ``ablation`` the ladder of earlier kernel designs.  Importing this package loads nothing;
the library is loaded on first use and a missing build raises.
"""
__all__ = ["ofhip"]
