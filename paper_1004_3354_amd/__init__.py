"""MI355X-native exact-diagonalization hot path: matrix-free spin-factorised H.v
and Lanczos for fixed-(N_up, N_dn) sectors of Hubbard and impurity Hamiltonians.

Importing the package loads nothing; ``paper_1004_3354_amd.ed`` binds the HIP
C-ABI library and raises if it is missing.
"""
__all__ = ["ed", "models", "workloads"]
