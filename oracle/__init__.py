"""Plain FP64 CPU oracle of the GDSW preconditioner (test infrastructure only:
imported by the test suite, the smoke check and the benchmark's CPU-baseline
leg; never by the GPU library)."""
