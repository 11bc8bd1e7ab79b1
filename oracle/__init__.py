"""FP64 CPU oracle for the scaled-ILU smoother (test infrastructure only)."""
