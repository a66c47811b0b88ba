"""CPU oracle of the p-bit sweep (test infrastructure only; see oracle.py)."""
