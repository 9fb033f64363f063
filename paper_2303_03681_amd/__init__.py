"""MI355X-native MPS-VQE energy evaluation: HIP kernels behind a C ABI.

The library (csrc/, built into libmps_hip.so) applies ansatz gates to a
matrix product state by two-site contraction and truncated one-sided Jacobi
SVD, restores the canonical form, and evaluates every Pauli string of a
Jordan-Wigner Hamiltonian by transfer-matrix products on the GPU's matrix
cores.  ``binding`` is the ctypes layer over include/mps.h.
"""

from .binding import Mps, MpsError, PauliSum, jacobi_svd, load, selftest_mfma

__all__ = ["Mps", "MpsError", "PauliSum", "jacobi_svd", "load", "selftest_mfma"]
