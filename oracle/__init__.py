"""FP64 CPU oracle: test infrastructure only (see ``lrnr_oracle``)."""
