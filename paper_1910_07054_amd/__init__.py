"""MI355X-native hybrid-FFT demagnetization field on non-equidistant layers.

The compute path lives in the HIP library ``libhfd.so`` (sources in
``csrc/``, C ABI declared in ``include/hfd.h``); ``hfd`` is its Python binding.
Importing this package loads nothing; ``hfd`` loads the library on first use
and raises if it has not been built.
"""
