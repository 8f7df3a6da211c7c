"""CPU float64 oracle (test infrastructure only; see psl_oracle)."""
