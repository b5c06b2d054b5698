"""MI355X-native hot path of the KPM / Chebyshev spectral method (KITE, arXiv:1910.05194).

The computation lives in the HIP library libkpm.so (C ABI in include/kpm.h);
``paper_1910_05194_amd.kpm`` is its thin ctypes binding.  Importing the
binding fails loudly when the library has not been built.
"""
