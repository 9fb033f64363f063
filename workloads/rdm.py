"""Jordan-Wigner expansions of reduced-density-matrix elements.

The fragment 1-RDM gamma_pq = <a+_p a_q> and 2-RDM
Gamma_pqrs = <a+_p a+_q a_r a_s> (spin orbitals, the conventions of
hamiltonian.py) are what a DMET loop takes from each fragment's VQE state
(Methods, "Density matrix embedding theory").  Each element is a monomial of
ladder operators whose JW expansion sum_k v_k P_k has complex v_k; since
every <P_k> is real, Re<M> = sum Re(v_k) <P_k> and Im<M> = sum Im(v_k) <P_k>.
This module lists, for a set of elements, the union of their strings and two
CSR rows per element (Re, Im) over that union.  It holds no MPS arithmetic.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .hamiltonian import PauliSum, _expand_monomials, _masks_to_codes, _n_words


@dataclass
class RdmRows:
    """Strings (a PauliSum with unit coefficients) and CSR rows: row 2e is
    Re<element e>, row 2e + 1 is Im<element e>."""

    strings: PauliSum
    row_ptr: np.ndarray   # (2 E + 1,) int64
    cols: np.ndarray      # (nnz,) int64
    vals: np.ndarray      # (nnz,) float64
    elements: np.ndarray  # (E, k) spin-orbital indices of each element


def _rows(n_qubits, orbs, daggers, drop=1e-14):
    words = _n_words(n_qubits)
    E = orbs[0].size
    keys, vals = _expand_monomials(orbs, daggers, np.ones(E, complex), words)
    elem = np.tile(np.arange(E), keys.shape[0] // max(E, 1))
    # unique strings over all elements
    kv = np.ascontiguousarray(keys).view(np.dtype((np.void, keys.dtype.itemsize * keys.shape[1]))).ravel()
    uniq, first, col = np.unique(kv, return_index=True, return_inverse=True)
    # combine repeats of one string within one element
    pair = elem.astype(np.int64) * uniq.size + col
    up, inv = np.unique(pair, return_inverse=True)
    re = np.bincount(inv, weights=vals.real, minlength=up.size)
    im = np.bincount(inv, weights=vals.imag, minlength=up.size)
    e_of, c_of = up // uniq.size, up % uniq.size
    rows_e, rows_c, rows_v, rows_r = [], [], [], []
    for part, v in ((0, re), (1, im)):
        keep = np.abs(v) > drop
        rows_r.append(2 * e_of[keep] + part)
        rows_c.append(c_of[keep])
        rows_v.append(v[keep])
    r = np.concatenate(rows_r)
    c = np.concatenate(rows_c)
    v = np.concatenate(rows_v)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    # keep only strings some row uses; renumber columns
    used = np.unique(c)
    remap = np.full(uniq.size, -1, np.int64)
    remap[used] = np.arange(used.size)
    c = remap[c]
    codes = _masks_to_codes(keys[first[used]], n_qubits, words)
    row_ptr = np.zeros(2 * E + 1, np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return PauliSum(n_qubits, codes, np.ones(used.size)), row_ptr, c.astype(np.int64), v


def one_rdm_rows(n_qubits: int) -> RdmRows:
    """Every element gamma_pq, p, q < n_qubits, in row-major order."""
    p, q = np.meshgrid(np.arange(n_qubits), np.arange(n_qubits), indexing="ij")
    p, q = p.ravel(), q.ravel()
    ps, rp, c, v = _rows(n_qubits, [p, q], [True, False])
    return RdmRows(ps, rp, c, v, np.stack([p, q], axis=1))


def two_rdm_rows(n_qubits: int) -> RdmRows:
    """Elements Gamma_pqrs with p < q and r < s (the others follow from
    antisymmetry), ordered by (p, q) then (r, s)."""
    pairs = [(a, b) for a in range(n_qubits) for b in range(a + 1, n_qubits)]
    el = np.array([(a, b, c, d) for (a, b) in pairs for (c, d) in pairs], dtype=np.int64)
    ps, rp, c, v = _rows(n_qubits, [el[:, 0], el[:, 1], el[:, 2], el[:, 3]], [True, True, False, False])
    return RdmRows(ps, rp, c, v, el)
