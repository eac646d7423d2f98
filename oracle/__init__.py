"""FP64 CPU oracle for two-component CVS-ADC(2) -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The GPU library never imports, calls or links it.
"""
