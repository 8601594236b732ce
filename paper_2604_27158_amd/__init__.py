"""MI355X (gfx950) hot path of the hybrid Fourier Neural Operator - Lattice Boltzmann
method: HIP kernels behind the C ABI of include/lbmfno.h, a ctypes binding
(lbmfno), seeded synthetic workloads (workloads) and the hybrid driver.

Importing the package loads nothing; the binding loads liblbmfno.so on first use
and raises if it (or a GPU) is missing.
"""
__all__ = ["lbmfno", "workloads"]
