"""FP64 CPU oracle of the BTDF-IB-LBM step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package. It shares no code with the HIP library.
"""
