"""One-sided Jacobi oracle: TEST INFRASTRUCTURE ONLY (see oracle.py)."""
