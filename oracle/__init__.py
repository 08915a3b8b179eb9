"""FP64 CPU oracle of the batched 2D physics step (test infrastructure only)."""
