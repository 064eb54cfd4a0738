"""CPU oracle for SZ dual-quantisation - TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. The GPU library never calls it.
"""
