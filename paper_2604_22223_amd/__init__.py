"""libqgw: one GW iteration on a tight-binding lattice, HIP kernels for gfx950.

The compute path lives in the C-ABI shared library ``libqgw.so`` (built from
``csrc/``); ``qgw`` is its thin ctypes binding.  ``workloads`` generates seeded
model inputs.  Importing this package does not load the library.
"""
