"""MI355X-native overlap-save variable-bandwidth filtering with HFSO coefficients.

The compute path is the HIP library ``libvbw.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/vbw.h``; ``vbw`` is its thin Python binding.
Importing this package loads nothing; the library is loaded on first use.
"""
