"""Energy gradients of the UCCSD ansatz by the parameter-shift rule, with
circuit-prefix caching, on the library's gates and expectations.

The ansatz is a product of Pauli exponentials U_k = exp(i phi_k P_k) with
phi_k = theta_j(k) c_k (Methods, "Unitary coupled cluster"; first-order
Trotter).  Since P_k^2 = 1, E as a function of one phi_k is
a + b cos(2 phi_k) + d sin(2 phi_k), so dE/dphi_k = E(phi_k + pi/4) -
E(phi_k - pi/4) exactly, and by the chain rule

    dE/dtheta_j = sum over k with j(k) = j of c_k [E(phi_k + pi/4) - E(phi_k - pi/4)].

Both shifted circuits of factor k share the gates of factors 0..k-1: one
handle keeps the state after that prefix and advances by one factor at a
time; each shifted evaluation copies it (mps_copy), applies the shifted
factor and the unchanged suffix, and measures the energy.  Up to `batch`
factors are evaluated together, their 2*batch gate lists in shared launches
(mps_apply_gates_multi) when the bonds allow it and their energies in one
pass (mps_expect_pauli_sum_multi).  Exact for a circuit whose
gates do not truncate; with truncation it is the shift rule applied to the
truncated circuit.
"""

from __future__ import annotations

import math

import numpy as np

from workloads.circuits import fuse_gates, pack_gates, pauli_exponential_gates, uccsd_exponentials

from . import binding


def _packed(code, phi, n):
    g = fuse_gates(pauli_exponential_gates(code, phi), n)
    if not g:
        return (np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 32), np.float64))
    q0, q1, u = pack_gates(g)
    return q0, q1, u.reshape(len(q0), -1)


def _cat(parts):
    q0 = np.concatenate([p[0] for p in parts]).astype(np.int32)
    q1 = np.concatenate([p[1] for p in parts]).astype(np.int32)
    u = np.concatenate([p[2] for p in parts]).reshape(len(q0), -1)
    return q0, q1, u


class ExponentialGradient:
    """E(theta) and dE/dtheta of a product of Pauli exponentials
    prod_k exp(i theta_j(k) c_k P_k), given as (j, codes, c) per factor in
    circuit order, for one Pauli sum."""

    def __init__(self, n_qubits: int, exps, plan: "binding.PauliSum", max_bond: int,
                 cutoff: float = 1e-14, bits=None, prec: str = "c128", batch: int = 8,
                 stream: int | None = None, n_params: int | None = None):
        self.n = int(n_qubits)
        self.exps = list(exps)
        self.n_params = n_params if n_params is not None else 1 + max((j for j, _, _ in self.exps), default=-1)
        self.plan = plan
        self.prec = prec
        self.batch = max(1, int(batch))
        self.bits = bits
        mk = lambda: binding.Mps(n_qubits, max_bond, cutoff, bits=bits, stream=stream)  # noqa: E731
        self.prefix = mk()
        self.work = [mk() for _ in range(2 * self.batch)]
        self.evaluations = 0
        self.gates_applied = 0

    def close(self):
        for m in [self.prefix] + self.work:
            m.close()

    def _segments(self, theta):
        seg, plus, minus = [], [], []
        for j, code, c in self.exps:
            phi = float(theta[j] * c)
            seg.append(_packed(code, phi, self.n))
            plus.append(_packed(code, phi + math.pi / 4, self.n))
            minus.append(_packed(code, phi - math.pi / 4, self.n))
        return seg, plus, minus

    def energy(self, theta) -> float:
        seg, _, _ = self._segments(np.asarray(theta, float))
        m = self.prefix
        m.reset(self.bits)
        q0, q1, u = _cat(seg)
        m.apply_gates(q0, q1, u)
        self.evaluations += 1
        self.gates_applied += len(q0)
        return m.expect(self.plan, self.prec)

    def energy_and_gradient(self, theta):
        theta = np.asarray(theta, float)
        if theta.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {theta.size}")
        seg, plus, minus = self._segments(theta)
        K = len(seg)
        # suffix k = segments k+1 .. K-1, as views of one concatenation
        full = _cat(seg) if K else _cat([_packed(np.zeros(self.n, np.uint8), 0.0, self.n)])
        off = np.zeros(K + 1, np.int64)
        for k in range(K):
            off[k + 1] = off[k] + len(seg[k][0])
        grad = np.zeros(self.n_params)
        self.prefix.reset(self.bits)
        multi_ok = True
        for k0 in range(0, K, self.batch):
            ks = list(range(k0, min(K, k0 + self.batch)))
            lists, handles = [], []
            for i, k in enumerate(ks):
                suffix = tuple(a[off[k + 1]:] for a in full)
                for s, shifted in enumerate((plus[k], minus[k])):
                    h = self.work[2 * i + s]
                    h.copy_from(self.prefix)
                    lists.append(_cat([shifted, suffix]))
                    handles.append(h)
                q0, q1, u = seg[k]
                if len(q0):
                    self.prefix.apply_gates(q0, q1, u)
                    self.gates_applied += len(q0)
            if multi_ok:
                try:
                    binding.apply_gates_multi(handles, lists)
                except binding.MpsError as e:
                    if e.name != "MPS_ERR_ARG" or any(int(x) for x in getattr(e, "n_done", [0])):
                        raise
                    multi_ok = False  # bonds beyond the batched limit: one handle at a time
            if not multi_ok:
                for h, l in zip(handles, lists):
                    h.apply_gates(*l)
            self.gates_applied += sum(len(l[0]) for l in lists)
            # the 2 * batch energies in one pass (launches shared by the handles)
            es = binding.expect_multi(handles, [self.plan] * len(handles), self.prec)
            for i, k in enumerate(ks):
                j, _, c = self.exps[k]
                grad[j] += c * (es[2 * i] - es[2 * i + 1])
            self.evaluations += 2 * len(ks)
        # the prefix handle now holds the whole circuit
        e = self.prefix.expect(self.plan, self.prec)
        self.evaluations += 1
        return e, grad


class UccsdGradient(ExponentialGradient):
    """E(theta) and dE/dtheta of (windowed) UCCSD for one Pauli sum."""

    def __init__(self, n_qubits: int, n_electrons: int, plan: "binding.PauliSum", max_bond: int,
                 cutoff: float = 1e-14, bits=None, window: int | None = None, prec: str = "c128",
                 batch: int = 8, stream: int | None = None):
        super().__init__(n_qubits, uccsd_exponentials(n_qubits, n_electrons, window), plan, max_bond,
                         cutoff, bits, prec, batch, stream)


def gradient_descent(grad: ExponentialGradient, theta0, steps: int, lr: float):
    """Plain steepest descent theta <- theta - lr dE/dtheta; returns the
    parameters and the energy before each step and after the last."""
    theta = np.array(theta0, float)
    energies = []
    for _ in range(steps):
        e, g = grad.energy_and_gradient(theta)
        energies.append(e)
        theta = theta - lr * g
    energies.append(grad.energy(theta))
    return theta, energies
