"""MI355X-native Harmonic Decomposition Factorization (HDF) hot path.

``paper_2202_03655_amd.hdf`` binds the C ABI of ``include/hdf.h`` (library
``paper_2202_03655_amd/lib/libhdf.so``, built by ``__graft_entry__.build()``).
"""
from .hdf import (CrossFactor, Factor, HDFError, HDFMatvec, build, plan_chebyshev,  # noqa: F401
                  plan_compress_cross, plan_cores, plan_degree, plan_index_set, HDF_FP64, HDF_MIXED)
