"""Plain FP64 CPU reference for the PSFD solve: test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package; the product path never does.
"""
