"""MI355X X-engine for the FX correlator of arXiv 1904.07778.

The compute path is the HIP library ``libxeng.so`` (gfx950 kernels behind
the C ABI in ``include/xeng.h``); ``paper_1904_07778_amd.xeng`` is its thin
ctypes binding with the same entry-point names.  Import of the binding
fails loudly when the library has not been built.
"""
__all__ = ["xeng"]
