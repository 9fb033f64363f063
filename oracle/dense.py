"""Dense statevector reference (test infrastructure).

The amplitude tensor c_{i1...iN} of Methods Eq. (mps) stored as a numpy array
of shape (2,)*N, axis q = qubit q = MPS site q+1 (so qubit 0 is the most
significant bit of the flat index).  Gates act by tensordot; a Pauli string
P(x, z) = i^{|x&z|} X^x Z^z acts on a basis state |b> as
i^{|x&z|} (-1)^{|z&b|} |b xor x>.
"""

from __future__ import annotations

import math

import numpy as np


def dense_zero_state(n: int) -> np.ndarray:
    psi = np.zeros((2,) * n, dtype=complex)
    psi[(0,) * n] = 1.0
    return psi


def dense_product_state(bits) -> np.ndarray:
    bits = [int(b) for b in bits]
    psi = np.zeros((2,) * len(bits), dtype=complex)
    psi[tuple(bits)] = 1.0
    return psi


def dense_apply_gate(psi: np.ndarray, q0: int, q1: int, u: np.ndarray) -> np.ndarray:
    """1q gate (q1 < 0) or 2q gate on (q0, q0+1) with row index 2*i_q0 + i_q1."""
    if q1 < 0:
        out = np.tensordot(u, psi, axes=([1], [q0]))  # new axis 0
        return np.moveaxis(out, 0, q0)
    assert q1 == q0 + 1
    u4 = np.asarray(u).reshape(2, 2, 2, 2)
    out = np.tensordot(u4, psi, axes=([2, 3], [q0, q1]))
    return np.moveaxis(out, [0, 1], [q0, q1])


def dense_apply_gates(psi: np.ndarray, gates) -> np.ndarray:
    for g in gates:
        psi = dense_apply_gate(psi, g.q0, g.q1, g.u)
    return psi


def _masks(code: np.ndarray):
    n = code.size
    x = 0
    z = 0
    for q in range(n):
        c = int(code[q])
        bit = 1 << (n - 1 - q)  # qubit q is the most significant for q = 0
        if c in (1, 2):
            x |= bit
        if c in (2, 3):
            z |= bit
    return x, z


def dense_apply_pauli(psi: np.ndarray, code: np.ndarray) -> np.ndarray:
    n = psi.ndim
    flat = psi.reshape(-1)
    x, z = _masks(np.asarray(code))
    idx = np.arange(flat.size, dtype=np.int64)
    parity = np.zeros(flat.size, dtype=np.int64)
    zz = idx & z
    while np.any(zz):
        parity ^= zz & 1
        zz >>= 1
    ny = bin(x & z).count("1")
    phase = (1j ** ny) * (1 - 2 * parity)
    out = np.empty_like(flat)
    out[idx ^ x] = phase * flat
    return out.reshape((2,) * n)


def dense_expect_pauli(psi: np.ndarray, code: np.ndarray) -> complex:
    return complex(np.vdot(psi.reshape(-1), dense_apply_pauli(psi, code).reshape(-1)))


def dense_energy(psi: np.ndarray, codes: np.ndarray, coeffs: np.ndarray) -> float:
    """<psi|H|psi>/<psi|psi>, summed exactly rounded (math.fsum)."""
    norm2 = float(np.vdot(psi.reshape(-1), psi.reshape(-1)).real)
    terms = [float(c) * dense_expect_pauli(psi, code).real for code, c in zip(codes, coeffs)]
    return math.fsum(terms) / norm2


_P1 = {
    0: np.eye(2, dtype=complex),
    1: np.array([[0, 1], [1, 0]], dtype=complex),
    2: np.array([[0, -1j], [1j, 0]], dtype=complex),
    3: np.array([[1, 0], [0, -1]], dtype=complex),
}


def dense_pauli_matrix(code: np.ndarray) -> np.ndarray:
    """Kronecker product of the string's 2x2 matrices (qubit 0 leftmost)."""
    m = np.ones((1, 1), dtype=complex)
    for c in code:
        m = np.kron(m, _P1[int(c)])
    return m


# --------------------------------------------------------------------------
# reduced density matrices by ladder operators (Methods, "Density matrix
# embedding theory": the fragment RDMs the embedding loop needs)
# --------------------------------------------------------------------------

def dense_annihilate(psi: np.ndarray, j: int) -> np.ndarray:
    """a_j psi for spin orbital j = qubit j under Jordan-Wigner: the occupied
    component (bit j = 1) moves to bit j = 0 with sign (-1)^(occupations of
    qubits 0..j-1)."""
    n = psi.ndim
    out = np.zeros_like(psi)
    src = [slice(None)] * n
    dst = [slice(None)] * n
    src[j] = 1
    dst[j] = 0
    sub = psi[tuple(src)]  # axes: every qubit but j
    if j > 0:
        occ = np.indices((2,) * j).sum(axis=0)  # occupations of qubits < j
        sign = (1 - 2 * (occ % 2)).reshape((2,) * j + (1,) * (n - 1 - j))
        sub = sub * sign
    out[tuple(dst)] = sub
    return out


def dense_rdm1(psi: np.ndarray) -> np.ndarray:
    """gamma_pq = <a+_p a_q> = (a_p psi)^+ (a_q psi) / <psi|psi>."""
    n = psi.ndim
    a = [dense_annihilate(psi, j).reshape(-1) for j in range(n)]
    nrm = np.vdot(psi.reshape(-1), psi.reshape(-1)).real
    return np.array([[np.vdot(a[p], a[q]) for q in range(n)] for p in range(n)]) / nrm


def dense_rdm2(psi: np.ndarray) -> np.ndarray:
    """Gamma_pqrs = <a+_p a+_q a_r a_s> = (a_q a_p psi)^+ (a_r a_s psi) / <psi|psi>."""
    n = psi.ndim
    two = {}
    for x in range(n):
        ax = dense_annihilate(psi, x)
        for y in range(n):
            two[(y, x)] = dense_annihilate(ax, y).reshape(-1)  # a_y a_x psi
    nrm = np.vdot(psi.reshape(-1), psi.reshape(-1)).real
    g = np.zeros((n, n, n, n), dtype=complex)
    for p in range(n):
        for q in range(n):
            bra = two[(q, p)]
            for r in range(n):
                for s in range(n):
                    g[p, q, r, s] = np.vdot(bra, two[(r, s)])
    return g / nrm
