"""MI355X-native layered-media FMM for the reflected field g_2^t (arXiv 1902.08250).

The compute path is the HIP library ``liblmfmm.so`` behind the C ABI declared in
``include/lmfmm.h``; ``paper_1902_08250_amd.lmfmm`` is its thin ctypes binding.
The library is loaded on first use, and every entry point raises if it is
missing: there is no CPU fallback.
"""
