"""Test infrastructure: the plain FP64 CPU oracle of the SCA block method (see sca_oracle)."""
