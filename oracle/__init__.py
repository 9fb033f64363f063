"""FP64 CPU oracle for the MPS-VQE energy evaluation -- TEST INFRASTRUCTURE.

This package is the plain, slow reference that the HIP library is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path (the C ABI library and its Python
binding) never does, and shares no code with it.

Contents
  dense    statevector definition: gates applied to the 2^N vector, Pauli
           strings applied by bit flip and phase; 1- and 2-RDMs from ladder
           operators applied to the vector.  With no truncation the MPS
           method reaches this result exactly (up to rounding).
  jacobi   one-sided (Hestenes) Jacobi SVD, Algorithm 1 of the paper, written
           for complex matrices.
  mps      the right-canonical MPS of Methods "MPS algorithm for quantum
           circuit simulation": one-qubit gates (Eq. 1q), two-qubit gates by
           the two-site contraction, lambda scaling, SVD and truncation
           (Eqs. C, C~, svd, Bl), re-canonicalisation, Pauli-string
           expectations by transfer matrices (Eqs. expec1, expec2) and the
           exactly rounded energy sum.

Parity pins (tests/test_oracle_*.py) tie every function to something other
than itself: dense brute force, closed forms, LAPACK, sum rules and the
variational bound.
"""

from .dense import (
    dense_zero_state,
    dense_product_state,
    dense_apply_gate,
    dense_apply_gates,
    dense_apply_pauli,
    dense_expect_pauli,
    dense_energy,
    dense_pauli_matrix,
    dense_annihilate,
    dense_rdm1,
    dense_rdm2,
)
from .jacobi import one_sided_jacobi_svd
from .mps import MpsOracle

__all__ = [
    "dense_zero_state",
    "dense_annihilate",
    "dense_rdm1",
    "dense_rdm2",
    "dense_product_state",
    "dense_apply_gate",
    "dense_apply_gates",
    "dense_apply_pauli",
    "dense_expect_pauli",
    "dense_energy",
    "dense_pauli_matrix",
    "one_sided_jacobi_svd",
    "MpsOracle",
]
