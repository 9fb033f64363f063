"""Right-canonical MPS in FP64 complex (test infrastructure).

Follows Methods "MPS algorithm for quantum circuit simulation" and "The
implementation of UCCSD with matrix product states":

  * state: c_{i1..iN} = B^{i1} B^{i2} ... B^{iN} (Eq. mps) with trivial outer
    bonds; sites 0..N-1 here, site q = qubit q; B[q] has shape
    (2, D_q, D_{q+1}) and lam[b] holds the singular values of bond b
    (bond b sits left of site b; lam[0] = lam[N] = [1]);
  * gauge: right-canonical, sum_s B^s B^{s+} = 1 (Eq. rc);
  * one-qubit gate: B^s <- sum_s' Q_{ss'} B^{s'} (Eq. 1q);
  * two-qubit gate on (q, q+1), the Hastings scheme: C = Q . (B_q B_{q+1})
    (Eq. C), C~ = lam_q C (Eq. C~), SVD C~ = U lam~ V (Eq. svd),
    B~_q = C V^+ (Eq. Bl), B~_{q+1} = V, lam_{q+1} <- lam~;
  * truncation (the paper: drop small singular values or keep the largest
    few): keep k = min(D, #{sigma_j > cutoff * ||sigma||_2}), k >= 1, then
    renormalise so the stored state has unit norm (lam~ and B~_q divided by
    ||sigma_1..k||); the discarded weight sum_{j>k} sigma_j^2 / sum sigma_j^2
    is accumulated;
  * expectations (Eqs. expec1, expec2): a string with support [m, n] starts
    from L = diag(lam_m^2), is carried through every site m..n by
    L <- sum_{ss'} sigma_{ss'} B^{s+} L B^{s'} and closed by a trace, the
    right boundary being the identity in right-canonical form;
  * energy: math.fsum of c_k Re<P_k>, i.e. exactly rounded.

The SVD of the two-qubit step is LAPACK's (numpy.linalg.svd); Algorithm 1
(oracle.jacobi) can be selected instead with ``svd="jacobi"``.

Re-canonicalisation is not spelled out in the paper; it is what restores the
right-canonical condition and exact Schmidt values that the lam^2 shortcut of
Eq. (expec1) relies on after truncation: a left-to-right Householder QR sweep
(numpy.linalg.qr) followed by a right-to-left SVD sweep.
"""

from __future__ import annotations

import math

import numpy as np

from .jacobi import one_sided_jacobi_svd

_PAULI = {
    0: np.eye(2, dtype=complex),
    1: np.array([[0, 1], [1, 0]], dtype=complex),
    2: np.array([[0, -1j], [1j, 0]], dtype=complex),
    3: np.array([[1, 0], [0, -1]], dtype=complex),
}


class MpsOracle:
    def __init__(self, n_qubits: int, max_bond: int, cutoff: float = 1e-14, bits=None,
                 svd: str = "lapack", canon_cutoff: float = 1e-14):
        self.n = int(n_qubits)
        self.max_bond = int(max_bond)
        self.cutoff = float(cutoff)
        self.canon_cutoff = float(canon_cutoff)
        self.svd = svd
        self.discarded = 0.0
        self.norm_before_canon = 1.0
        self.reset(bits)

    # ------------------------------------------------------------------ state
    def reset(self, bits=None):
        """Product state |b>: B_q^s = delta_{s, b_q} (1x1), all lam = [1]."""
        bits = np.zeros(self.n, dtype=int) if bits is None else np.asarray(bits, dtype=int)
        self.B = []
        for q in range(self.n):
            t = np.zeros((2, 1, 1), dtype=complex)
            t[int(bits[q]), 0, 0] = 1.0
            self.B.append(t)
        self.lam = [np.ones(1) for _ in range(self.n + 1)]
        self.discarded = 0.0
        self.canonical = True

    def bond_dims(self):
        return [1] + [self.B[q].shape[2] for q in range(self.n)]

    # ------------------------------------------------------------------ gates
    def apply_1q(self, q: int, u: np.ndarray):
        """Eq. (1q)."""
        self.B[q] = np.einsum("st,tab->sab", np.asarray(u, dtype=complex), self.B[q])

    def _svd(self, m: np.ndarray):
        if self.svd == "jacobi":
            u, s, v = one_sided_jacobi_svd(m)
            return u, s, v.conj().T
        return np.linalg.svd(m, full_matrices=False)

    def apply_2q(self, q: int, u: np.ndarray):
        """Hastings scheme on bond q+1: Eqs. (C), (C~), (svd), (Bl)."""
        Bl, Br = self.B[q], self.B[q + 1]
        dl, dr = Bl.shape[1], Br.shape[2]
        # Eq. (C): C^{t1 t2}_{l r} = sum_{m, s1, s2} Q^{t1 t2}_{s1 s2} B^{s1}_{l m} B^{s2}_{m r}
        theta = np.einsum("alm,bmr->ablr", Bl, Br)
        q4 = np.asarray(u, dtype=complex).reshape(2, 2, 2, 2)
        C = np.einsum("cdab,ablr->cdlr", q4, theta)
        Cmat = C.transpose(0, 2, 1, 3).reshape(2 * dl, 2 * dr)  # rows (t1, l), cols (t2, r)
        # Eq. (C~): row scaling by lam of the bond left of site q
        lam_l = self.lam[q]
        Ct = (np.tile(lam_l, 2)[:, None]) * Cmat
        _, s, vh = self._svd(Ct)
        norm = math.sqrt(float(np.sum(s * s)))
        keep = int(np.sum(s > self.cutoff * norm))
        k = max(1, min(self.max_bond, keep))
        kept = math.sqrt(float(np.sum(s[:k] ** 2)))
        if norm > 0:
            self.discarded += float(np.sum(s[k:] ** 2)) / (norm * norm)
        vk = vh[:k]  # (k, 2 dr): rows of V, cols (t2, r)
        # Eq. (Bl): B~_q = C V^+ ; B~_{q+1} = V
        newl = (Cmat @ vk.conj().T) / kept  # (2 dl, k) rows (t1, l)
        self.B[q] = newl.reshape(2, dl, k)
        self.B[q + 1] = vk.reshape(k, 2, dr).transpose(1, 0, 2).copy()
        self.lam[q + 1] = s[:k] / kept
        self.canonical = False

    def apply_gate(self, q0: int, q1: int, u: np.ndarray):
        if q1 < 0:
            self.apply_1q(q0, u)
        else:
            assert q1 == q0 + 1, "only nearest-neighbour two-qubit gates"
            self.apply_2q(q0, u)

    def apply_gates(self, gates):
        for g in gates:
            self.apply_gate(g.q0, g.q1, g.u)

    # ------------------------------------------------------------ canonical
    def canonicalize(self):
        """Left-to-right QR sweep, then right-to-left SVD sweep.

        Afterwards every B is right-canonical, every lam holds the Schmidt
        values of its bond (round-off zeros below canon_cutoff*||s|| dropped)
        and the state has unit norm; the norm it had before is recorded.
        """
        n = self.n
        carry = np.ones((1, 1), dtype=complex)
        A = []
        for q in range(n):
            M = np.einsum("ab,sbc->sac", carry, self.B[q])  # (2, r, Dr)
            r = M.shape[1]
            Q, R = np.linalg.qr(M.reshape(2 * r, M.shape[2]))
            A.append(Q.reshape(2, r, Q.shape[1]))
            carry = R
        A[-1] = np.einsum("sab,bc->sac", A[-1], carry)  # carry is (r, 1)
        carry = np.ones((A[-1].shape[2], 1), dtype=complex)
        newB = [None] * n
        lam = [None] * (n + 1)
        lam[n] = np.ones(1)
        for q in range(n - 1, -1, -1):
            M = np.einsum("sab,bc->asc", A[q], carry)  # (Dl, 2, r)
            dl, r = M.shape[0], M.shape[2]
            U, S, Vh = np.linalg.svd(M.reshape(dl, 2 * r), full_matrices=False)
            tot = math.sqrt(float(np.sum(S * S)))
            k = max(1, int(np.sum(S > self.canon_cutoff * tot)))
            newB[q] = Vh[:k].reshape(k, 2, r).transpose(1, 0, 2).copy()
            lam[q] = S[:k]
            carry = U[:, :k] * S[:k][None, :]
        norm = float(lam[0][0])
        self.norm_before_canon = norm
        for b in range(n):
            lam[b] = lam[b] / math.sqrt(float(np.sum(lam[b] ** 2)))
        lam[0] = np.ones(1)
        self.B = newB
        self.lam = lam
        self.canonical = True
        return norm

    # ---------------------------------------------------------- expectations
    def expect_pauli(self, code) -> complex:
        """Eq. (expec2): lam^2 open at the first non-identity site, transfer
        through every site of the support, trace at the last one."""
        code = np.asarray(code)
        sup = np.nonzero(code)[0]
        if sup.size == 0:
            return complex(np.sum(self.lam[0] ** 2))
        m, n = int(sup[0]), int(sup[-1])
        L = np.diag(self.lam[m] ** 2).astype(complex)
        for q in range(m, n + 1):
            L = self._transfer(L, q, int(code[q]))
        return complex(np.trace(L))

    def _transfer(self, L, q, c):
        """L <- sum_{ss'} sigma_{ss'} B^{s+} L B^{s'}."""
        B = self.B[q]
        sig = _PAULI[c]
        out = np.zeros((B.shape[2], B.shape[2]), dtype=complex)
        for s in range(2):
            for sp in range(2):
                if sig[s, sp] != 0:
                    out += sig[s, sp] * (B[s].conj().T @ L @ B[sp])
        return out

    def expect_pauli_full(self, code) -> complex:
        """Same expectation from the full contraction: identity transfers from
        the left boundary and an explicit right boundary (no gauge assumed),
        divided by the norm."""
        code = np.asarray(code)
        L = np.ones((1, 1), dtype=complex)
        N = np.ones((1, 1), dtype=complex)
        for q in range(self.n):
            L = self._transfer(L, q, int(code[q]))
            N = self._transfer(N, q, 0)
        return complex(L[0, 0] / N[0, 0])

    def expect_terms(self, codes) -> np.ndarray:
        return np.array([self.expect_pauli(c) for c in codes])

    def energy(self, codes, coeffs) -> float:
        """E = sum_k c_k Re<P_k> over a canonical state, exactly rounded."""
        if not self.canonical:
            self.canonicalize()
        vals = [float(c) * self.expect_pauli(code).real for code, c in zip(codes, coeffs)]
        return math.fsum(vals)

    # ------------------------------------------------------------- helpers
    def to_statevector(self) -> np.ndarray:
        psi = np.ones((1, 1), dtype=complex)  # (amplitudes, bond)
        for q in range(self.n):
            B = self.B[q]
            psi = np.einsum("pa,sab->psb", psi, B).reshape(-1, B.shape[2])
        return psi.reshape((2,) * self.n)

    def right_canonical_residual(self) -> float:
        r = 0.0
        for B in self.B:
            g = np.einsum("sab,scb->ac", B, B.conj())
            r = max(r, float(np.max(np.abs(g - np.eye(g.shape[0])))))
        return r

    def norm2(self) -> float:
        N = np.ones((1, 1), dtype=complex)
        for q in range(self.n):
            N = self._transfer(N, q, 0)
        return float(N[0, 0].real)
