"""FP64 CPU oracle of the PORTA hot path -- test infrastructure only (see oracle.py)."""
