"""Oracle package: a plain CPU float64 reference of the D-bar method.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the CPU-baseline leg of the benchmark.
The GPU library never imports it, and it imports nothing from the GPU library.
"""
