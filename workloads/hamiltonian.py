"""Random-integral electronic Hamiltonians and their Jordan-Wigner Pauli sums.

The electronic Hamiltonian in second quantisation (Methods, "Unitary coupled
cluster") is turned into a qubit operator sum_k c_k P_k by the Jordan-Wigner
map; the energy evaluation then measures every P_k.  The paper takes its
integrals from PySCF; here they are seeded random numbers with the symmetry
of real molecular integrals.

Conventions (the paper fixes none of them):
  * spatial integrals: h_pq real symmetric, (pq|rs) in chemists' notation with
    the 8-fold permutational symmetry of real orbitals;
  * spin orbitals interleaved, j = 2p + sigma (sigma = 0 alpha, 1 beta);
  * H = sum_{pq,s} h_pq a+_{ps} a_{qs}
        + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs};
  * Jordan-Wigner: a+_j = Z_0 ... Z_{j-1} (X_j - i Y_j) / 2;
  * qubit j is site j+1 of the MPS; no nuclear-repulsion constant.

Pauli strings are handled in the symplectic form P(x, z) = i^{|x & z|} X^x Z^z
with bit j of the masks standing for qubit j, stored as ``words`` uint64
words so that 100-qubit strings fit.
"""

from __future__ import annotations

import os
from dataclasses import dataclass
from math import comb

import numpy as np

CODE_I, CODE_X, CODE_Y, CODE_Z = 0, 1, 2, 3


@dataclass
class PauliSum:
    """sum_k coeffs[k] * P_k with codes[k, q] in {0:I, 1:X, 2:Y, 3:Z}."""

    n_qubits: int
    codes: np.ndarray  # (T, n_qubits) uint8
    coeffs: np.ndarray  # (T,) float64

    @property
    def n_terms(self) -> int:
        return int(self.coeffs.shape[0])

    def subset(self, idx) -> "PauliSum":
        idx = np.asarray(idx)
        return PauliSum(self.n_qubits, np.ascontiguousarray(self.codes[idx]),
                        np.ascontiguousarray(self.coeffs[idx]))


# --------------------------------------------------------------------------
# integrals
# --------------------------------------------------------------------------

def _pair_index(p, q):
    return p * (p + 1) // 2 + q if p >= q else q * (q + 1) // 2 + p


def random_integrals(n_s: int, rng: np.random.Generator, h_std: float = 0.5,
                     g_std: float = 0.1):
    """h (n_s x n_s) symmetric and g = (pq|rs) (n_s^4) with 8-fold symmetry.

    Draw order: h's upper triangle with diagonal, row-major; then one value per
    8-fold orbit of g in canonical order (p>=q, r>=s, pq>=rs with pq the
    compound pair index), looping over pq then rs <= pq.
    """
    h = np.zeros((n_s, n_s))
    iu = np.triu_indices(n_s)
    hv = rng.normal(0.0, h_std, size=iu[0].size)
    h[iu] = hv
    h[iu[1], iu[0]] = hv

    pairs = [(p, q) for p in range(n_s) for q in range(p + 1)]
    npair = len(pairs)
    a_idx, b_idx = np.tril_indices(npair)  # a >= b, row-major: pq then rs <= pq
    gv = rng.normal(0.0, g_std, size=a_idx.size)
    P = np.array(pairs, dtype=np.int64)
    p, q = P[a_idx, 0], P[a_idx, 1]
    r, s = P[b_idx, 0], P[b_idx, 1]
    g = np.zeros((n_s,) * 4)
    for (i, j, k, l) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                         (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
        g[i, j, k, l] = gv
    return h, g


# --------------------------------------------------------------------------
# symplectic Pauli algebra on uint64 word masks
# --------------------------------------------------------------------------

def _n_words(n_qubits: int) -> int:
    return (n_qubits + 63) // 64


def _bit_masks(j: np.ndarray, words: int):
    """(len(j), words) uint64 with only bit j set."""
    out = np.zeros((j.size, words), dtype=np.uint64)
    w = j // 64
    b = (j % 64).astype(np.uint64)
    out[np.arange(j.size), w] = np.left_shift(np.uint64(1), b)
    return out


def _below_masks(j: np.ndarray, words: int):
    """(len(j), words) uint64 with bits 0 .. j-1 set (the Jordan-Wigner Z tail)."""
    out = np.zeros((j.size, words), dtype=np.uint64)
    full = np.uint64(0xFFFFFFFFFFFFFFFF)
    for w in range(words):
        lo = 64 * w
        nb = np.clip(j - lo, 0, 64)
        col = np.where(nb >= 64, full,
                       np.left_shift(np.uint64(1), (nb % 64).astype(np.uint64)) - np.uint64(1))
        col = np.where(nb <= 0, np.uint64(0), col)
        out[:, w] = col
    return out


def _popcount(m: np.ndarray) -> np.ndarray:
    return np.bitwise_count(m).sum(axis=-1).astype(np.int64)


def _pauli_mul(x1, z1, x2, z2):
    """P(x1,z1) P(x2,z2) = i^e P(x1^x2, z1^z2); returns (x, z, e mod 4)."""
    x3 = x1 ^ x2
    z3 = z1 ^ z2
    e = _popcount(x1 & z1) + _popcount(x2 & z2) + 2 * _popcount(z1 & x2) - _popcount(x3 & z3)
    return x3, z3, np.mod(e, 4)


_I_POW = np.array([1.0, 1.0j, -1.0, -1.0j])


def _expand_monomials(orbs, daggers, coef, words):
    """Jordan-Wigner expansion of sum_t coef[t] * prod_k ladder(orbs[k][t]).

    ``orbs`` is a list of int arrays (one per ladder operator, left to right),
    ``daggers`` the matching creation flags.  Returns (keys, values) where keys
    are (T', 2*words) uint64 rows [x | z] and values complex coefficients.
    """
    nops = len(orbs)
    T = coef.size
    bits = [_bit_masks(o, words) for o in orbs]
    below = [_below_masks(o, words) for o in orbs]
    keys, vals = [], []
    for choice in range(1 << nops):
        x = np.zeros((T, words), dtype=np.uint64)
        z = np.zeros((T, words), dtype=np.uint64)
        e = np.zeros(T, dtype=np.int64)
        fac = np.full(T, 1.0 + 0.0j)
        for k in range(nops):
            c = (choice >> k) & 1
            xk = bits[k]
            zk = below[k] | bits[k] if c else below[k]
            # a+_j = (P(e_j, zlt) - i P(e_j, zlt|e_j)) / 2 ;  a_j with +i
            if c:
                fac = fac * ((-0.5j) if daggers[k] else (0.5j))
            else:
                fac = fac * 0.5
            x, z, de = _pauli_mul(x, z, xk, zk)
            e = e + de
        fac = fac * _I_POW[np.mod(e, 4)] * coef
        keys.append(np.concatenate([x, z], axis=1))
        vals.append(fac)
    return np.concatenate(keys, axis=0), np.concatenate(vals)


def _reduce(keys, vals):
    """Combine like Pauli strings."""
    if keys.shape[0] == 0:
        return keys, vals
    keys = np.ascontiguousarray(keys)
    v = keys.view(np.dtype((np.void, keys.dtype.itemsize * keys.shape[1]))).ravel()
    uniq, inv = np.unique(v, return_inverse=True)
    re = np.bincount(inv, weights=vals.real, minlength=uniq.size)
    im = np.bincount(inv, weights=vals.imag, minlength=uniq.size)
    ukeys = keys[np.unique(inv, return_index=True)[1]]
    return ukeys, re + 1j * im


def _masks_to_codes(keys, n_qubits, words):
    x = keys[:, :words]
    z = keys[:, words:]
    codes = np.zeros((keys.shape[0], n_qubits), dtype=np.uint8)
    for q in range(n_qubits):
        w, b = divmod(q, 64)
        xb = (x[:, w] >> np.uint64(b)) & np.uint64(1)
        zb = (z[:, w] >> np.uint64(b)) & np.uint64(1)
        # (x,z): (0,0) I, (1,0) X, (1,1) Y, (0,1) Z
        codes[:, q] = np.where(xb == 1, np.where(zb == 1, CODE_Y, CODE_X),
                               np.where(zb == 1, CODE_Z, CODE_I)).astype(np.uint8)
    return codes


def _two_body_chunk(args):
    """JW expansion of the two-body terms with first orbital p0, like strings combined."""
    p0, g, words = args
    n_s = g.shape[0]
    q, r, s_, sg, tg = np.meshgrid(np.arange(n_s), np.arange(n_s), np.arange(n_s),
                                   np.arange(2), np.arange(2), indexing="ij")
    q, r, s_, sg, tg = (a.ravel() for a in (q, r, s_, sg, tg))
    j1 = 2 * p0 + sg
    j2 = 2 * r + tg
    j3 = 2 * s_ + tg
    j4 = 2 * q + sg
    keep = (j1 != j2) & (j3 != j4)
    coef = 0.5 * g[p0, q, r, s_]
    keep &= coef != 0.0
    if not np.any(keep):
        return None, None
    k2, v2 = _expand_monomials([j1[keep], j2[keep], j3[keep], j4[keep]],
                               [True, True, False, False],
                               coef[keep].astype(complex), words)
    return _reduce(k2, v2)


_WORKER: dict = {}


def _init_two_body(g, words):
    _WORKER["g"] = g
    _WORKER["words"] = words


def _two_body_worker(p0):
    return _two_body_chunk((p0, _WORKER["g"], _WORKER["words"]))


def jw_hamiltonian(h: np.ndarray, g: np.ndarray, drop_rel: float = 1e-15,
                   workers: int | None = None, progress=None) -> PauliSum:
    """Jordan-Wigner Pauli sum of the spin-orbital Hamiltonian built from (h, g).

    Like strings are combined; only round-off residues |c| < drop_rel*max|c|
    are dropped.  Coefficients of a Hermitian operator are real; the imaginary
    parts are checked to vanish.
    """
    n_s = h.shape[0]
    n = 2 * n_s
    words = _n_words(n)
    acc_k, acc_v = [], []

    # one-body: h_pq a+_{p s} a_{q s}
    p, q, s = np.meshgrid(np.arange(n_s), np.arange(n_s), np.arange(2), indexing="ij")
    p, q, s = p.ravel(), q.ravel(), s.ravel()
    coef = h[p, q].astype(complex)
    k1, v1 = _expand_monomials([2 * p + s, 2 * q + s], [True, False], coef, words)
    acc_k.append(k1)
    acc_v.append(v1)

    # two-body, chunked over p: 1/2 (pq|rs) a+_{p s} a+_{r t} a_{s' t} a_{q s};
    # chunks are independent (optionally in worker processes) and concatenated
    # in p order, so the result does not depend on the number of workers
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if n_s >= 30 else 1
    args = [(p0, g, words) for p0 in range(n_s)]
    say = progress or (lambda msg: None)
    if workers > 1:
        # fresh interpreters ("spawn"), not forks: the caller may already hold
        # a GPU context, which a forked child must not inherit
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        parts = []
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                 initializer=_init_two_body, initargs=(g, words)) as ex:
            for i, part in enumerate(ex.map(_two_body_worker, range(n_s))):
                parts.append(part)
                say(f"two-body chunk {i + 1}/{n_s}")
    else:
        parts = [_two_body_chunk(a) for a in args]
    say("combining like strings")
    for k2, v2 in parts:
        if k2 is not None:
            acc_k.append(k2)
            acc_v.append(v2)

    keys, vals = _reduce(np.concatenate(acc_k), np.concatenate(acc_v))
    scale = np.max(np.abs(vals)) if vals.size else 0.0
    if scale > 0:
        assert np.max(np.abs(vals.imag)) <= 1e-12 * max(1.0, scale), "non-Hermitian JW sum"
    keep = np.abs(vals) > drop_rel * scale
    keys, vals = keys[keep], vals[keep].real.copy()
    codes = _masks_to_codes(keys, n, words)
    # deterministic, readable order: by support start, then lexicographic codes
    order = np.lexsort(codes.T[::-1])
    return PauliSum(n, np.ascontiguousarray(codes[order]), np.ascontiguousarray(vals[order]))


def generic_term_count(n_s: int) -> int:
    """Number of distinct JW strings for generic real integrals (interleaved spins).

    identity + Z_j + Z_iZ_j + same-spin hops (bare or with one Z toggled)
    + opposite-spin double hops (4 strings per orbital-pair pair) + same-spin
    double hops (12 of the 16 even-Y patterns per orbital quadruple survive:
    antisymmetry makes two patterns per spin cancel).
    """
    n = 2 * n_s
    return (1 + n + comb(n, 2) + 4 * comb(n_s, 2) * (n - 1)
            + 4 * comb(n_s, 2) ** 2 + 12 * comb(n_s, 4))


def sample_terms(psum: PauliSum, count: int, rng: np.random.Generator) -> PauliSum:
    """Uniform sample without replacement of ``count`` distinct strings (kept in order)."""
    if count >= psum.n_terms:
        return psum
    idx = np.sort(rng.choice(psum.n_terms, size=count, replace=False))
    return psum.subset(idx)


def hf_bits(n_qubits: int, n_electrons: int) -> np.ndarray:
    """Hartree-Fock bitstring: spin orbitals 0 .. n_electrons-1 occupied."""
    bits = np.zeros(n_qubits, dtype=np.uint8)
    bits[:n_electrons] = 1
    return bits
