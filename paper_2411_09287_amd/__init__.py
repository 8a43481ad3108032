"""MI355X-native three-party secure linear evaluation over Z_{2^64} (arXiv 2411.09287).

The compute path is the C-ABI library ``libmpc3.so`` (HIP kernels for gfx950),
declared in ``include/mpc3.h``; ``paper_2411_09287_amd.mpc3`` is its thin ctypes
binding.  ``workloads`` holds the seeded synthetic inputs.
"""
