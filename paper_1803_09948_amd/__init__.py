"""MI355X-native Helmholtz FMM / BIE / GMRES (arXiv 1803.09948 hot path).

The compute path is the HIP library `_lib/libhfmm.so` (built by
`paper_1803_09948_amd.build`); `hfmm` is its thin ctypes binding.  Importing
this package does not load the library; the first call into `hfmm` does, and
fails loudly if it has not been built.
"""
__all__ = ["hfmm"]
