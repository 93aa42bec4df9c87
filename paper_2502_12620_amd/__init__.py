"""MI355X-native block-based AMR explicit DG (compressible Euler) library.

The compute path is the HIP library ``libdgamr.so`` behind the C-ABI in
``include/dgamr.h``; ``dgamr`` is its thin Python binding.
"""
