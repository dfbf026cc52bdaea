"""MI355X (gfx950) synchronous parallel simulated annealing.

The library ``libsa_hip.so`` (C ABI in ``include/sa.h``) runs the whole
annealing on the GPU; ``sa`` is its Python binding.
"""
