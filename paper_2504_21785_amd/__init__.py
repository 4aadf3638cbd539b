"""MI355X-native reconstruction of frozen Gaussian wave-packets (direct sum and FGGC).

The compute path lives in the HIP library ``libfggc.so`` (sources in ``csrc/``,
C ABI in ``include/fggc.h``); ``fggc`` is the thin ctypes binding and
``workloads`` the seeded synthetic input generator.  Importing this package
does not load the library: ``paper_2504_21785_amd.fggc`` does, and fails
loudly when it has not been built.
"""
