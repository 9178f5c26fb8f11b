"""FP64 CPU oracle of the ChiSao per-cycle update (test infrastructure only)."""
