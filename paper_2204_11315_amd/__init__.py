"""Compressed out-of-core 3-D stencil sweeps on MI355X (gfx950).

The compute path lives in the HIP/C++ shared library built from `csrc/`
(C ABI declared in include/oc.h); `oc` is its thin ctypes binding.
"""
