"""Plain FP64 CPU oracle of the TDDFT hot path (test infrastructure only)."""
