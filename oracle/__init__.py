"""FP64 CPU oracle for the LSKUM sweep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls into it.
"""
