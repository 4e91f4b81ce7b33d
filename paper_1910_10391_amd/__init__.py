"""MI355X-native radiation integrals (arXiv:1910.10391, Sec. II and IV).

``paper_1910_10391_amd.rad`` is the Python binding of the C-ABI library
``librad.so`` (hand-written HIP kernels for gfx950); ``paper_1910_10391_amd.synth``
holds the seeded input generators.  Importing this package loads neither.
"""
__all__ = ["rad", "synth"]
