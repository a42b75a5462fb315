"""FP64 CPU oracle of the HLBM step -- test infrastructure only.

Imported by tests/, by the smoke check and by the benchmark's CPU-baseline
leg; never by the product path."""
