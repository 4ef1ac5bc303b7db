"""hyeig: the hybrid eigensolver hot path of arXiv 2305.15552 for MI355X.

The computation lives in ``libhyeig.so`` (HIP kernels for gfx950 and host C++
behind the C-ABI of ``include/hyeig.h``).  ``paper_2305_15552_amd.hyeig`` is the
ctypes binding; importing it loads the library and fails if it is not built.
"""
