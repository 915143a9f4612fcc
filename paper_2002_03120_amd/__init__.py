"""MI355X-native SDPD-DEM hot path (arXiv 2002.03120): HIP kernels behind a C ABI."""
