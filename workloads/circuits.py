"""Gate lists for the UCCSD and hardware-efficient ansatze.

A gate list is the contract shared by the oracle and the HIP library: both
apply exactly the same sequence of one-qubit gates (2x2) and nearest-neighbour
two-qubit gates (4x4, row index 2*i_q0 + i_q1 with q1 = q0 + 1).

UCCSD (Methods, "Unitary coupled cluster" and "The implementation of UCCSD
with matrix product states"): each excitation generator theta (tau - tau^+) is
Jordan-Wigner mapped to i * sum_k c_k P_k with mutually commuting strings, and
first-order Trotterisation turns the ansatz into a product of Pauli
exponentials exp(i theta c_k P_k).  Each exponential is compiled to a basis
change, a nearest-neighbour parity ladder, a Z rotation and the inverse
ladder; identity qubits inside the support are crossed by SWAPs so that the
parity skips them.

Hardware-efficient ansatz (Results, "Peak performance"; Discussions): layers
of Ry/Rz on every qubit followed by CNOTs on every neighbouring pair
(brickwork: even pairs, then odd pairs).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .hamiltonian import (
    CODE_I, CODE_X, CODE_Y, CODE_Z, _expand_monomials, _masks_to_codes,
    _n_words, _reduce,
)


@dataclass
class Gate:
    q0: int
    q1: int  # -1 for a one-qubit gate, else q0 + 1
    u: np.ndarray  # (2,2) or (4,4) complex


_SQ2 = 1.0 / np.sqrt(2.0)


def gate_h():
    return np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=complex)


def gate_sdg():
    return np.array([[1, 0], [0, -1j]], dtype=complex)


def gate_rx(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=complex)


def gate_ry(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return np.array([[c, -s], [s, c]], dtype=complex)


def gate_rz(t):
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=complex)


def gate_cnot():
    """Control q0, target q1 (row index 2*i_q0 + i_q1)."""
    m = np.eye(4, dtype=complex)
    m[2:, 2:] = [[0, 1], [1, 0]]
    return m


def gate_swap():
    m = np.zeros((4, 4), dtype=complex)
    m[0, 0] = m[3, 3] = 1
    m[1, 2] = m[2, 1] = 1
    return m


# --------------------------------------------------------------------------
# Pauli exponentials
# --------------------------------------------------------------------------

def pauli_exponential_gates(code: np.ndarray, phi: float) -> list[Gate]:
    """Nearest-neighbour gates for exp(i phi P), P given by per-qubit codes."""
    code = np.asarray(code)
    sup = np.nonzero(code)[0]
    if sup.size == 0:
        return []  # global phase only
    m, n = int(sup[0]), int(sup[-1])
    pre, post = [], []
    for q in sup:
        c = int(code[q])
        if c == CODE_X:
            pre.append(Gate(int(q), -1, gate_h()))
            post.append(Gate(int(q), -1, gate_h()))
        elif c == CODE_Y:
            b = gate_h() @ gate_sdg()  # maps Y to Z: b Y b^+ = Z
            pre.append(Gate(int(q), -1, b))
            post.append(Gate(int(q), -1, b.conj().T))
    ladder = []
    for q in range(m, n):
        if code[q + 1] != CODE_I:
            ladder.append(Gate(q, q + 1, gate_cnot()))
        else:
            ladder.append(Gate(q, q + 1, gate_swap()))
    rot = Gate(n, -1, np.diag([np.exp(1j * phi), np.exp(-1j * phi)]).astype(complex))
    return pre + ladder + [rot] + ladder[::-1] + post


# --------------------------------------------------------------------------
# UCCSD
# --------------------------------------------------------------------------

def uccsd_excitations(n_qubits: int, n_electrons: int):
    """Spin-conserving singles (i, a) then doubles (i, j, a, b), lexicographic.

    Spin orbital j has spin j % 2; occupied = 0 .. n_electrons-1.
    """
    occ = range(n_electrons)
    vir = range(n_electrons, n_qubits)
    singles = [(i, a) for i in occ for a in vir if i % 2 == a % 2]
    doubles = []
    for i in occ:
        for j in occ:
            if j <= i:
                continue
            for a in vir:
                for b in vir:
                    if b <= a:
                        continue
                    if sorted((i % 2, j % 2)) == sorted((a % 2, b % 2)):
                        doubles.append((i, j, a, b))
    return singles, doubles


def _generator_strings(n_qubits, orbs_left, orbs_right):
    """JW strings of tau - tau^+ with tau = a+_{l0} [a+_{l1}] a_{r0} [a_{r1}].

    Returns (codes, c) with tau - tau^+ = i * sum_k c_k P_k.
    """
    words = _n_words(n_qubits)
    ops = list(orbs_left) + list(orbs_right)
    dag = [True] * len(orbs_left) + [False] * len(orbs_right)
    one = np.ones(1, dtype=complex)
    k1, v1 = _expand_monomials([np.array([o]) for o in ops], dag, one, words)
    # tau^+ = reversed product with daggers flipped
    ops_h = ops[::-1]
    dag_h = [not d for d in dag[::-1]]
    k2, v2 = _expand_monomials([np.array([o]) for o in ops_h], dag_h, -one, words)
    keys, vals = _reduce(np.concatenate([k1, k2]), np.concatenate([v1, v2]))
    keep = np.abs(vals) > 1e-14
    keys, vals = keys[keep], vals[keep]
    assert np.max(np.abs(vals.real)) < 1e-14, "generator must be anti-Hermitian"
    codes = _masks_to_codes(keys, n_qubits, words)
    return codes, vals.imag.copy()


def window_excitations(n_qubits: int, n_electrons: int, window: int = 5):
    """UCCSD excitations whose spatial orbitals all lie within `window`
    consecutive orbitals (Methods, ansatz for hydrogen chains: operators built
    on every 5 consecutive orbitals)."""
    singles, doubles = uccsd_excitations(n_qubits, n_electrons)
    def ok(*spin_orbitals):
        sp = [o // 2 for o in spin_orbitals]
        return max(sp) - min(sp) < window
    return [e for e in singles if ok(*e)], [e for e in doubles if ok(*e)]


def gsd_window_excitations(n_qubits: int, window: int = 5):
    """Generalised singles and doubles (any orbitals, not only occupied to
    virtual; spin-conserving) whose spatial orbitals lie within `window`
    consecutive orbitals, i.e. inside one of the windows starting at every
    orbital (Methods, ansatz for hydrogen chains).  Singles (p, q), p > q:
    a+_p a_q; doubles (p, q, r, s), p > q, r > s, (p, q) > (r, s):
    a+_p a+_q a_r a_s.  Each generator tau - tau^+ appears once."""
    def ok(*so):
        sp = [o // 2 for o in so]
        return max(sp) - min(sp) < window
    singles = [(p, q) for p in range(n_qubits) for q in range(p)
               if p % 2 == q % 2 and ok(p, q)]
    pairs = [(p, q) for p in range(n_qubits) for q in range(p)]
    doubles = []
    for (p, q) in pairs:
        for (r, s) in pairs:
            if (r, s) >= (p, q):
                continue
            if sorted((p % 2, q % 2)) != sorted((r % 2, s % 2)):
                continue
            if ok(p, q, r, s):
                doubles.append((p, q, r, s))
    return singles, doubles


def qubit_adapt_pool(n_qubits: int, window: int = 5) -> np.ndarray:
    """Operator pool of the windowed qubit-ADAPT ansatz: the JW strings of
    every windowed GSD generator with all Z letters removed, strings with an
    even number of Y dropped (the Hamiltonian is real), duplicates merged.
    Returns codes (P, n_qubits) uint8 in lexicographic order."""
    singles, doubles = gsd_window_excitations(n_qubits, window)
    rows = []
    for (p, q) in singles:
        codes, _ = _generator_strings(n_qubits, (p,), (q,))
        rows.append(codes)
    for (p, q, r, s) in doubles:
        codes, _ = _generator_strings(n_qubits, (p, q), (r, s))
        rows.append(codes)
    if not rows:
        return np.zeros((0, n_qubits), np.uint8)
    codes = np.concatenate(rows).copy()
    codes[codes == CODE_Z] = CODE_I
    odd_y = (np.sum(codes == CODE_Y, axis=1) % 2) == 1
    codes = np.unique(codes[odd_y], axis=0)
    return np.ascontiguousarray(codes[np.lexsort(codes.T[::-1])], dtype=np.uint8)


def uccsd_exponentials(n_qubits: int, n_electrons: int, window: int | None = None):
    """The Pauli exponentials of first-order Trotterised UCCSD in circuit
    order: a list of (parameter index j, string codes, c) for the factors
    exp(i theta_j c P)."""
    if window is None:
        singles, doubles = uccsd_excitations(n_qubits, n_electrons)
    else:
        singles, doubles = window_excitations(n_qubits, n_electrons, window)
    exc = [((a,), (i,)) for (i, a) in singles] + [((a, b), (i, j)) for (i, j, a, b) in doubles]
    out = []
    for j, (left, right) in enumerate(exc):
        codes, c = _generator_strings(n_qubits, left, right)
        for code, ck in zip(codes, c):
            out.append((j, code, float(ck)))
    return out


def uccsd_gates(n_qubits: int, n_electrons: int, theta: np.ndarray, window: int | None = None) -> list[Gate]:
    """First-order Trotterised UCCSD: prod_ex prod_k exp(i theta_ex c_k P_k).
    With `window`, only the excitations of window_excitations are used."""
    theta = np.asarray(theta, dtype=float)
    n_par = uccsd_n_params(n_qubits, n_electrons, window)
    assert theta.size == n_par, (theta.size, n_par)
    gates: list[Gate] = []
    for j, code, ck in uccsd_exponentials(n_qubits, n_electrons, window):
        gates.extend(pauli_exponential_gates(code, float(theta[j] * ck)))
    return gates


def uccsd_n_params(n_qubits: int, n_electrons: int, window: int | None = None) -> int:
    if window is None:
        s, d = uccsd_excitations(n_qubits, n_electrons)
    else:
        s, d = window_excitations(n_qubits, n_electrons, window)
    return len(s) + len(d)


# --------------------------------------------------------------------------
# hardware-efficient brickwork
# --------------------------------------------------------------------------

def brickwork_gates(n_qubits: int, angles: np.ndarray) -> list[Gate]:
    """angles[l, q] = (ry, rz): per layer Ry then Rz on every qubit, then
    CNOT(q, q+1) for even q, then for odd q (control = lower index)."""
    gates: list[Gate] = []
    for layer in angles:
        for q in range(n_qubits):
            gates.append(Gate(q, -1, gate_ry(layer[q, 0])))
            gates.append(Gate(q, -1, gate_rz(layer[q, 1])))
        for start in (0, 1):
            for q in range(start, n_qubits - 1, 2):
                gates.append(Gate(q, q + 1, gate_cnot()))
    return gates


# --------------------------------------------------------------------------
# gate-list simplification (exact: products of the given matrices)
# --------------------------------------------------------------------------

def fuse_gates(gates: list[Gate], n_qubits: int) -> list[Gate]:
    """Merge consecutive 1q gates, fold them into the next 2q gate on that
    qubit, merge consecutive 2q gates on the same pair and drop identities.
    The product of the returned list equals the product of the input."""
    pending: list[np.ndarray | None] = [None] * n_qubits
    out: list[Gate] = []
    last2: list[int] = [-1] * n_qubits  # index in out of last 2q gate touching q

    def flush(q):
        if pending[q] is not None:
            if not np.allclose(pending[q], np.eye(2), atol=1e-15):
                out.append(Gate(q, -1, pending[q]))
                last2[q] = -1
            pending[q] = None

    for g in gates:
        if g.q1 < 0:
            pending[g.q0] = g.u if pending[g.q0] is None else g.u @ pending[g.q0]
            continue
        a, b = g.q0, g.q1
        u = g.u
        ua = pending[a] if pending[a] is not None else np.eye(2)
        ub = pending[b] if pending[b] is not None else np.eye(2)
        if pending[a] is not None or pending[b] is not None:
            u = u @ np.kron(ua, ub)
        pending[a] = pending[b] = None
        j = last2[a]
        if j >= 0 and j == last2[b] and out[j].q0 == a and out[j].q1 == b:
            m = u @ out[j].u
            out[j] = Gate(a, b, m)
            if np.allclose(m, np.eye(4), atol=1e-14):
                out[j] = None  # type: ignore[assignment]
                last2[a] = last2[b] = -1
            continue
        out.append(Gate(a, b, u))
        last2[a] = last2[b] = len(out) - 1
    for q in range(n_qubits):
        flush(q)
    return [g for g in out if g is not None]


def pack_gates(gates: list[Gate]):
    """Flat arrays for the C ABI: q0[int32], q1[int32], u (G, 16, 2) float64
    (2x2 gates occupy the first 4 entries)."""
    G = len(gates)
    q0 = np.array([g.q0 for g in gates], dtype=np.int32)
    q1 = np.array([g.q1 for g in gates], dtype=np.int32)
    u = np.zeros((G, 16, 2), dtype=np.float64)
    for i, g in enumerate(gates):
        flat = np.asarray(g.u, dtype=complex).ravel()
        u[i, :flat.size, 0] = flat.real
        u[i, :flat.size, 1] = flat.imag
    return q0, q1, u
