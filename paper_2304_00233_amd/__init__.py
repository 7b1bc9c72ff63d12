"""MI355X-native fictitious-wave-domain CSEM FDTD hot path (libEMM method,
arXiv:2304.00233): HIP kernels behind a C ABI (include/emm.h) plus this thin
Python binding.  `from paper_2304_00233_amd import emm` loads the library."""
