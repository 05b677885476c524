"""MI355X-native batched simulation of stochastic cognitive models.

The compute path lives in ``libcm.so`` (HIP for gfx950 behind a C ABI,
``include/cm.h``); ``paper_2110_15425_amd.cm`` is its Python binding.
Importing this package loads nothing: the binding loads the library on
first use and fails loudly if it is missing.
"""
