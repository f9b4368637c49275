"""MI355X-native event-based Monte Carlo transport with thread-data remapping.

The compute path is the HIP library ``libmcx.so`` (C ABI declared in
``include/mcx.h``); ``paper_2506_00263_amd.mcx`` is its ctypes binding.
Importing this package loads nothing: ``inputs`` (seeded problem
generators) works without a GPU or a built library.
"""
__version__ = "0.1.0"
