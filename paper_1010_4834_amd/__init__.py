"""MI355X (gfx950) SU(2) lattice gauge Monte Carlo: checkerboard heat-bath
sweeps of the Wilson action and the plaquette, Polyakov-loop and APE-smeared
Wilson-loop measurements (Cardoso & Bicudo, arXiv:1010.4834).

The computation lives in libsu2.so (HIP kernels behind the C ABI of
include/su2.h); `paper_1010_4834_amd.su2` is its Python binding.
"""
__all__ = ["su2"]
