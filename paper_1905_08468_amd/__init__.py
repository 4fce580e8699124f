"""MUFFIN wideband deconvolution with ADA-PT tuning on AMD MI355X.

The compute path is the HIP library libmuffin.so (include/muffin.h);
``paper_1905_08468_amd.muffin`` is its ctypes binding.
"""
