"""Pyramidal Lucas-Kanade feature tracking on AMD Instinct MI355X (gfx950).

The work runs in the HIP kernels of ``liblkmi.so`` behind the C ABI of
``include/lk.h``; ``paper_2607_01757_amd.lk`` is its ctypes binding.
"""
__all__ = ["lk"]
