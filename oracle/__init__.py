"""Oracle: plain, slow, obviously correct CPU implementations of what the
generalized FrequencyHough path computes.  Test infrastructure only: the test
suite, the smoke check and the benchmark's CPU-baseline leg use it; the
product library never does."""
