"""Plain FP64 CPU oracle (test infrastructure only; see mot_oracle)."""
