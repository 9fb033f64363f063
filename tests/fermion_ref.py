"""Independent fermionic reference for the Jordan-Wigner pins.

Builds second-quantised operators as dense matrices by acting on occupation
number basis states with explicit sign counting (a_j |n> = (-1)^{sum_{k<j} n_k}
|n - e_j>), never through Pauli algebra.  Mode j is the most significant bit
of the basis index, matching the dense statevector convention.
"""

from __future__ import annotations

import numpy as np


def ladder(n: int, j: int, dagger: bool) -> np.ndarray:
    dim = 1 << n
    m = np.zeros((dim, dim))
    for b in range(dim):
        occ = (b >> (n - 1 - j)) & 1
        if dagger and occ:
            continue
        if not dagger and not occ:
            continue
        sign = 1.0
        for k in range(j):
            if (b >> (n - 1 - k)) & 1:
                sign = -sign
        out = b ^ (1 << (n - 1 - j))
        m[out, b] = sign
    return m


def hamiltonian_matrix(h: np.ndarray, g: np.ndarray) -> np.ndarray:
    n_s = h.shape[0]
    n = 2 * n_s
    cre = [ladder(n, j, True) for j in range(n)]
    ann = [ladder(n, j, False) for j in range(n)]
    H = np.zeros((1 << n, 1 << n))
    for p in range(n_s):
        for q in range(n_s):
            for s in range(2):
                H += h[p, q] * cre[2 * p + s] @ ann[2 * q + s]
    for p in range(n_s):
        for q in range(n_s):
            for r in range(n_s):
                for s_ in range(n_s):
                    v = 0.5 * g[p, q, r, s_]
                    if v == 0.0:
                        continue
                    for sg in range(2):
                        for tg in range(2):
                            H += v * (cre[2 * p + sg] @ cre[2 * r + tg]
                                      @ ann[2 * s_ + tg] @ ann[2 * q + sg])
    return H


def number_operator(n: int) -> np.ndarray:
    return sum(ladder(n, j, True) @ ladder(n, j, False) for j in range(n))


def sz_operator(n: int) -> np.ndarray:
    return sum((0.5 if j % 2 == 0 else -0.5) * ladder(n, j, True) @ ladder(n, j, False)
               for j in range(n))


def pauli_sum_matrix(codes, coeffs) -> np.ndarray:
    from oracle import dense_pauli_matrix
    n = codes.shape[1]
    M = np.zeros((1 << n, 1 << n), dtype=complex)
    for code, c in zip(codes, coeffs):
        M += c * dense_pauli_matrix(code)
    return M


def hf_energy_closed_form(h: np.ndarray, g: np.ndarray, n_electrons: int) -> float:
    """E_HF = sum_i h_ii + 1/2 sum_ij (<ij|ij> - <ij|ji>) over occupied spin orbitals."""
    occ = list(range(n_electrons))
    e = 0.0
    for i in occ:
        e += h[i // 2, i // 2]
    for i in occ:
        for j in occ:
            pi, pj = i // 2, j // 2
            e += 0.5 * g[pi, pi, pj, pj]
            if i % 2 == j % 2:
                e -= 0.5 * g[pi, pj, pj, pi]
    return e
