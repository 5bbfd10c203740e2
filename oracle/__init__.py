"""FP64 CPU oracle for the shifted-COCG solver (test infrastructure only)."""
