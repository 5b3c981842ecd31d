"""FP64 CPU oracle of the Gaussian-splatting hot path (test infrastructure only)."""
