"""MI355X-native scaled-ILU smoother (arXiv 2111.09512): HIP kernels behind a C-ABI."""
