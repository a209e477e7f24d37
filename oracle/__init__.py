"""EXACT CPU oracle (test infrastructure; see oracle/exact_oracle.c)."""
