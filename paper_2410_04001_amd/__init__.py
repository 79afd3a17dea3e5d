"""MI355X (gfx950) implementation of the LRNR / FastLRNR physics-informed hot
path (arXiv 2410.04001): HIP kernels behind the C ABI of include/lrnr.h.

Submodules: ``_clib`` (ctypes loader), ``api`` (torch wrappers),
``build_lib`` (in-tree build of liblrnr.so).
"""
