"""MI355X-native HashGPU hashing path.

``paper_1202_3669_amd.hashgpu`` is the ctypes binding of the C-ABI library
``libhashgpu.so`` (declared in ``include/hashgpu.h``); importing it loads the
library and raises if it has not been built.  ``paper_1202_3669_amd.inputs``
draws the seeded synthetic inputs.
"""
