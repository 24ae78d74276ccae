"""FP64 CPU oracle for the vdW-DF nonlocal correlation (test infrastructure only)."""
