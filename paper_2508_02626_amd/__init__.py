"""MI355X-native DA fast multipole method (arXiv 2508.02626): HIP kernels for
gfx950 behind the C ABI of include/fmm.h, with a thin Python binding.

Importing the package loads nothing; `paper_2508_02626_amd.fmm` loads the
library on first use and raises if it is missing.
"""
