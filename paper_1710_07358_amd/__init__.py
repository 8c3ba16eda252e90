"""MI355X-native parallel reduction (arXiv 1710.07358), HIP kernels behind a C ABI."""
