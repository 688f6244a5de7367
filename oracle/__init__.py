"""CPU oracle for the triangle-soup rasterization step.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark. The product path never imports it.
"""
