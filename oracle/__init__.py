"""FP64 CPU oracle of the nested continuation-value Monte Carlo.

Test infrastructure only: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.
"""
