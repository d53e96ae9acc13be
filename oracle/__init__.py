"""FP64 CPU oracle of the path tracer (test infrastructure only; never used by the product path)."""
