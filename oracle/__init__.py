"""FP64 CPU oracle (test infrastructure only; see fr_oracle.cpp)."""
