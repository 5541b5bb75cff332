"""Seeded synthetic workloads (inputs only, none of the method's
arithmetic): the populations and inputs that both the GPU library's
callers (tests, bench, smoke check) and the CPU oracle's tests use.  It
imports neither the library nor the oracle."""
