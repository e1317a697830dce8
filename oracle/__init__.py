"""CPU oracle of the LCG construction -- test infrastructure only (see oracle.py)."""
