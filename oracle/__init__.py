"""Serial CPU oracle and exact reference tools (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The product path never does.
"""
