"""FP64 CPU oracle of the forward render (test infrastructure only)."""
