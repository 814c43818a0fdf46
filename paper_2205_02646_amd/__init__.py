"""RL-JSDE reconstruction of three-quarter-sampling measurements on MI355X.

The hot path lives in ``libljsde.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/ljsde.h``); ``ljsde`` is its Python binding.
"""
