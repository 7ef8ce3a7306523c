"""CPU oracle for the fractal encoder (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path never does.
"""
