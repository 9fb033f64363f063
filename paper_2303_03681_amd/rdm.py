"""Fragment 1- and 2-RDMs of a device-resident MPS (the step after the energy
in the paper's DMET loop; Methods, "Density matrix embedding theory").

Every element's Jordan-Wigner strings are evaluated in one expectation pass
over their union (same tries, kernels and precisions as the energy), and the
elements are formed on the device as compensated linear combinations
(mps_expect_pauli_rows): Re and Im of each element are two rows.
"""

from __future__ import annotations

import numpy as np

from workloads.rdm import one_rdm_rows, two_rdm_rows

from . import binding


class RdmEvaluator:
    """gamma_pq = <a+_p a_q> and Gamma_pqrs = <a+_p a+_q a_r a_s> (spin
    orbitals = qubits) for MPSs of one qubit count."""

    def __init__(self, n_qubits: int, two_body: bool = True):
        self.n = int(n_qubits)
        self.r1 = one_rdm_rows(self.n)
        self.p1 = binding.PauliSum(self.r1.strings.codes, self.r1.strings.coeffs)
        self.r2 = two_rdm_rows(self.n) if two_body else None
        self.p2 = binding.PauliSum(self.r2.strings.codes, self.r2.strings.coeffs) if two_body else None

    def one_rdm(self, m: "binding.Mps", prec: str = "c128") -> np.ndarray:
        r = self.r1
        out = m.expect_rows(self.p1, r.row_ptr, r.cols, r.vals, prec)
        return (out[0::2] + 1j * out[1::2]).reshape(self.n, self.n)

    def two_rdm(self, m: "binding.Mps", prec: str = "c128") -> np.ndarray:
        if self.r2 is None:
            raise ValueError("built without the two-body rows")
        r = self.r2
        out = m.expect_rows(self.p2, r.row_ptr, r.cols, r.vals, prec)
        val = out[0::2] + 1j * out[1::2]
        n = self.n
        g = np.zeros((n, n, n, n), dtype=complex)
        p, q, s_, t = r.elements.T
        # antisymmetry in (p, q) and in (r, s); elements with p = q or r = s vanish
        g[p, q, s_, t] = val
        g[q, p, s_, t] = -val
        g[p, q, t, s_] = -val
        g[q, p, t, s_] = val
        return g
