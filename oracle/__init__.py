"""CPU FP64 oracle for RBE2D -- test infrastructure only (see oracle.py)."""
