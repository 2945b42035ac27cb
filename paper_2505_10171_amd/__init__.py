"""MI355X-native coupled colour-gradient LBM + DEM hot path (arXiv 2505.10171).

The compute path is the HIP library ``csrc/liblbm.so`` behind the C ABI declared in
``include/lbm.h``; :mod:`paper_2505_10171_amd.lbm` is its thin ctypes binding.
"""
