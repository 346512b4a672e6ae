"""MI355X-native p-multigrid gamma-cycle with cyclic-reduction line smoothers.

The compute path is the C-ABI library ``libpmg.so`` (hand-written HIP kernels
for gfx950); ``paper_2504_10710_amd.pmg`` is its thin ctypes binding.  Nothing
is loaded at import time, so ``paper_2504_10710_amd.inputs`` can be used on a
machine without the library.
"""
