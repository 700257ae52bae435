"""MI355X (gfx950) implementation of the GAPS-2 dipole parton shower
(arXiv:2511.19633): HIP kernels behind the C-ABI in include/gaps.h, with a thin
ctypes binding.  The package never falls back to a CPU path."""
