"""libhasf: homotopic alternating sequential filter (arXiv:1603.09337) on MI355X.

The compute path is the HIP library ``_lib/libhasf.so`` (C ABI, see
``include/libhasf.h``); ``paper_1603_09337_amd.hasf`` is its ctypes binding.
Importing this package loads nothing; importing ``hasf`` loads the library and
fails loudly when it is missing.
"""
