"""MI355X-native particle-tracking interpolation (libptk) and its Python binding.

The library (``libptk.so``, C ABI in ``include/ptk.h``) implements the hot path
of Lalescu, Bramas, Rampp & Wilczek's particle-tracking method: binning of
particles by grid cell, the tensor-product kernel interpolation of a periodic
3-component field (Sec. 2.2), its gradient, and the tracer time stepping.
``paper_2107_01104_amd.ptk`` is the binding; it requires the built library.
"""
