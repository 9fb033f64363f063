"""Pauli sums whose environment pool would not fit in device memory.

One plan keeps an environment (D x D) for every prefix and suffix node of its
tries; at 100 qubits and D = 512 the 2^20 sampled strings need about 2.2e5
nodes, 470 GB in complex64.  The strings are therefore sorted (so that shared
prefixes stay together) and cut into chunks of at most `max_strings`; each
chunk is one plan, evaluated on the same MPS with the same kernels by one
mps_expect_pauli_sums call: each chunk's compensated (sum, error) pair stays
on the device and the pairs are added there in chunk order.  The per-string
values are the same as from one plan up to the rounding order of their
transfer products.
"""

from __future__ import annotations

import numpy as np

from . import binding


class ChunkedPauliSum:
    def __init__(self, codes: np.ndarray, coeffs: np.ndarray, max_strings: int):
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        if codes.ndim != 2 or codes.shape[0] != coeffs.size:
            raise ValueError("codes must be (terms, qubits) with one coefficient per term")
        self.n_terms = coeffs.size
        self.order = np.lexsort(codes.T[::-1]) if self.n_terms else np.zeros(0, np.int64)
        step = max(1, int(max_strings))
        self.plans = []
        self.bounds = []
        for a in range(0, self.n_terms, step):
            idx = self.order[a:a + step]
            self.plans.append(binding.PauliSum(codes[idx], coeffs[idx]))
            self.bounds.append((a, min(self.n_terms, a + step)))

    def stats(self) -> list[dict]:
        return [p.stats() for p in self.plans]

    def expect(self, m: "binding.Mps", prec: str = "c128", per_term: bool = False):
        if not self.plans:
            return (0.0, np.zeros(0)) if per_term else 0.0
        if per_term:
            e, v = m.expect_chunks(self.plans, prec, per_term=True)
            per = np.zeros(self.n_terms)
            per[self.order] = v
            return e, per
        return m.expect_chunks(self.plans, prec)

    def close(self):
        for p in self.plans:
            p.close()
        self.plans = []
