"""MI355X-native batch-dynamic approximate k-core decomposition (PLDS).

The library lives in ``libplds.so`` (HIP kernels for gfx950 behind the C ABI of
``include/plds.h``); ``paper_2106_03824_amd.plds`` is its thin ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
