"""One-sided (Hestenes) Jacobi SVD -- Methods "SVD and one-side Jacobi",
Algorithm 1, generalised to complex matrices (test infrastructure).

Algorithm 1 sweeps over all column pairs (i, j), i < j, in cyclic order.  For
each pair it forms b_ii = a_i^+ a_i, b_jj = a_j^+ a_j, b_ij = a_i^+ a_j and, if
|b_ij| is not negligible against sqrt(b_ii b_jj), rotates the two columns of A
(and of V) by the Jacobi matrix J built from t and tau.  The sweep loop stops
when a whole sweep performs no rotation; then sigma_i = ||a_i||, u_i = a_i /
sigma_i and the triple is sorted by descending sigma.

Complex reading (the paper writes the real case): with b_ij = |b_ij| e^{i phi},
    tau = (b_ii - b_jj) / (2 |b_ij|),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
    c = 1 / sqrt(1 + t^2),  s = t c,   sign(0) = +1,
    J restricted to (i, j) = [[c, -s e^{i phi}], [s e^{-i phi}, c]],
which is the paper's real J when phi = 0 and makes the new columns exactly
orthogonal.  A rotation is skipped when |b_ij| <= eps sqrt(b_ii b_jj) or
|b_ij| <= eps^2 ||A||_F^2, with eps = m * 2^-53 by default (the paper leaves
eps open).  The absolute floor makes inner products that are pure round-off
count as zero: without it the surplus columns of a matrix with more columns
than rows, which converge to round-off-sized vectors, would keep rotating
among themselves and the sweep loop would never see a rotation-free sweep.
Columns whose norm is zero get a zero u_i (their sigma is 0).
"""

from __future__ import annotations

import math

import numpy as np


class JacobiNoConvergence(RuntimeError):
    pass


def one_sided_jacobi_svd(a: np.ndarray, eps: float | None = None, max_sweeps: int = 60,
                         return_sweeps: bool = False):
    """A (m x n) = U diag(sigma) V^+ by Algorithm 1; returns (U, sigma, V)."""
    A = np.array(a, dtype=complex, copy=True)
    m, n = A.shape
    V = np.eye(n, dtype=complex)
    if eps is None:
        eps = m * 2.0 ** -53
    floor = (eps * eps) * float(np.sum(np.abs(A) ** 2))
    sweeps = 0
    converged = False
    for _ in range(max_sweeps):
        sweeps += 1
        passed = True
        for i in range(n - 1):
            for j in range(i + 1, n):
                ai = A[:, i]
                aj = A[:, j]
                bii = float(np.vdot(ai, ai).real)
                bjj = float(np.vdot(aj, aj).real)
                bij = complex(np.vdot(ai, aj))
                mag = abs(bij)
                if mag <= floor or mag <= eps * math.sqrt(bii * bjj):
                    continue
                tau = (bii - bjj) / (2.0 * mag)
                sgn = 1.0 if tau >= 0.0 else -1.0
                t = sgn / (abs(tau) + math.sqrt(1.0 + tau * tau))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                e = bij / mag  # e^{i phi}
                new_i = c * ai + s * np.conj(e) * aj
                new_j = -s * e * ai + c * aj
                A[:, i] = new_i
                A[:, j] = new_j
                vi = V[:, i].copy()
                vj = V[:, j]
                V[:, i] = c * vi + s * np.conj(e) * vj
                V[:, j] = -s * e * vi + c * vj
                passed = False
        if passed:
            converged = True
            break
    if not converged:
        raise JacobiNoConvergence(f"no convergence after {max_sweeps} sweeps")
    sigma = np.sqrt(np.sum(np.abs(A) ** 2, axis=0))
    U = np.zeros_like(A)
    nz = sigma > 0
    U[:, nz] = A[:, nz] / sigma[nz]
    order = np.argsort(-sigma, kind="stable")
    out = (U[:, order], sigma[order], V[:, order])
    if return_sweeps:
        return out + (sweeps,)
    return out
