"""CPU oracle for the market split lattice method (test infrastructure only).

This package is the plain, slow, independent reference implementation that
the GPU library is checked against.  It may be imported only by the tests,
the smoke check and the benchmark's CPU-baseline leg; the product path never
imports it, and it imports nothing from the product package.
"""
