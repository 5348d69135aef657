"""MI355X-native arbitrary-precision ball dot products and matrix products.

The compute path is the C-ABI library ``libarbgpu.so`` (hand-written HIP for
gfx950); :mod:`paper_1901_04289_amd.arbgpu` is its thin Python binding.
Importing this package does not load the library.
"""
