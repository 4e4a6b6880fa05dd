"""FP64 CPU oracle for the APMGSRN hot path -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the HIP library.
"""
