"""MI355X-native H^2 hierarchical-matrix matrix-vector product.

The compute path is the HIP library ``libh2mv.so`` (C ABI, see
``include/h2mv.h``); :mod:`paper_1902_01829_amd.h2mv` is its thin ctypes
binding.  Importing this package loads nothing: import the binding to load
the library.
"""
