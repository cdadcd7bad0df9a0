"""MI355X-native CD-WAC core-level G0W0 self-energy.

The compute path is the HIP library ``libcdwac.so`` (hand-written gfx950
kernels behind a C ABI, declared in ``include/cdwac.h``); ``cdwac`` is its thin
ctypes binding.  ``synth`` and ``grids`` build the inputs.
"""
