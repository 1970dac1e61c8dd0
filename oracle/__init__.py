"""FP64 CPU oracle for the IHT hot path (test infrastructure only; see oracle.py)."""
