"""MI355X (gfx950) nested continuation-value Monte Carlo for multi-asset
Bermudan options (Doan et al., INRIA RR-6530, 2008).

The compute path is the HIP library libbmc.so (C ABI in include/bmc.h); the
`bmc` module is its ctypes binding and `inputs` generates seeded synthetic
option specs.
"""
__all__ = ["bmc", "inputs"]
