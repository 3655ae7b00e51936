"""MI355X (gfx950) Oriented FAST over an image pyramid.

The detector is the C-ABI library libof_hip.so (include/of.h); ``ofhip`` is its thin
Python binding, ``batch`` the graph-captured batched runner with its autotuner and
``serve`` the continuous-batching request loop.  Importing this package loads nothing;
the library is loaded on first use and a missing build raises.
"""
__all__ = ["ofhip"]
