"""Seeded synthetic workloads (inputs only) and search-quality metrics.

Shared by the tests, the benchmark and the smoke check.  Holds none of the
method's arithmetic: no encoding, no Delta, no top-k of proxy scores.
"""
