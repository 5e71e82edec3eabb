"""CPU oracle (test infrastructure only; see taylens_oracle.py)."""
