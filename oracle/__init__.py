"""CPU oracle (test infrastructure only; see oracle/gwn_oracle.c)."""
