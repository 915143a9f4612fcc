"""FP64 CPU oracle of the SDPD-DEM hot path (test infrastructure only)."""
