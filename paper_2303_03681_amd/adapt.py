"""Windowed qubit-ADAPT ansatz construction and the bond-dimension rule
(Methods, "The wave function ansatz for hydrogen chain simulations").

The pool is the Z-free, odd-Y JW strings of the generalised singles and
doubles inside windows of consecutive orbitals (workloads.qubit_adapt_pool).
Each ADAPT iteration measures, for every pool string P, the derivative of the
energy with respect to a new factor exp(i theta P) appended to the current
circuit, at theta = 0, by the parameter-shift rule:
E(exp(i pi/4 P) psi) - E(exp(-i pi/4 P) psi).  The string with the largest
|derivative| is appended, and all angles are then optimised by steepest
descent with parameter-shift gradients (gradients.ExponentialGradient).  The
pool derivatives run 2*batch handles at a time: copies of the current state
(mps_copy), the two shifted factors applied in shared launches
(mps_apply_gates_multi), then the energies.

The bond dimension is chosen as in the paper's D benchmark: energies over an
increasing list of D, and the first D_i with |E(D_i) - E(D_i+1)| below the
tolerance (1e-3 Ha there).
"""

from __future__ import annotations

import math

import numpy as np

from . import binding
from .gradients import ExponentialGradient, _cat, _packed


class QubitAdapt:
    def __init__(self, n_qubits: int, plan: "binding.PauliSum", pool: np.ndarray, max_bond: int,
                 cutoff: float = 1e-14, bits=None, prec: str = "c128", batch: int = 32,
                 stream: int | None = None):
        self.n = int(n_qubits)
        self.plan = plan
        self.pool = np.ascontiguousarray(pool, dtype=np.uint8)
        self.max_bond, self.cutoff, self.bits = max_bond, cutoff, bits
        self.prec, self.batch, self.stream = prec, max(1, int(batch)), stream
        self.ops: list[int] = []      # pool indices of the factors, in circuit order
        self.theta = np.zeros(0)
        mk = lambda: binding.Mps(n_qubits, max_bond, cutoff, bits=bits, stream=stream)  # noqa: E731
        self.state = mk()
        self.work = [mk() for _ in range(2 * self.batch)]
        self.history: list[dict] = []

    def close(self):
        for m in [self.state] + self.work:
            m.close()

    def _exps(self):
        return [(j, self.pool[a], 1.0) for j, a in enumerate(self.ops)]

    def prepare(self) -> float:
        """State of the current circuit at the current angles; its energy."""
        self.state.reset(self.bits)
        if self.ops:
            q0, q1, u = _cat([_packed(self.pool[a], float(t), self.n) for a, t in zip(self.ops, self.theta)])
            if len(q0):
                self.state.apply_gates(q0, q1, u)
        return self.state.expect(self.plan, self.prec)

    def pool_gradients(self) -> np.ndarray:
        """dE/dtheta at theta = 0 of appending exp(i theta P) for every pool string."""
        P = self.pool.shape[0]
        g = np.zeros(P)
        for a0 in range(0, P, self.batch):
            idx = list(range(a0, min(P, a0 + self.batch)))
            handles, lists = [], []
            for i, a in enumerate(idx):
                for s, sign in enumerate((1.0, -1.0)):
                    h = self.work[2 * i + s]
                    h.copy_from(self.state)
                    handles.append(h)
                    lists.append(_packed(self.pool[a], sign * math.pi / 4, self.n))
            try:
                binding.apply_gates_multi(handles, lists)
            except binding.MpsError as e:
                if e.name != "MPS_ERR_ARG" or any(int(x) for x in getattr(e, "n_done", [0])):
                    raise
                for h, l in zip(handles, lists):
                    h.apply_gates(*l)
            es = binding.expect_multi(handles, [self.plan] * len(handles), self.prec)
            for i, a in enumerate(idx):
                g[a] = es[2 * i] - es[2 * i + 1]
        return g

    def iterate(self, opt_steps: int = 5, lr: float = 0.1) -> dict:
        """One ADAPT iteration: select, append, optimise.  Returns its record."""
        e0 = self.prepare()
        g = self.pool_gradients()
        a = int(np.argmax(np.abs(g)))
        self.ops.append(a)
        self.theta = np.append(self.theta, 0.0)
        grad = ExponentialGradient(self.n, self._exps(), self.plan, self.max_bond, self.cutoff, self.bits,
                                   self.prec, batch=min(8, len(self.ops)), stream=self.stream)
        energies = []
        for _ in range(opt_steps):
            e, gr = grad.energy_and_gradient(self.theta)
            energies.append(e)
            self.theta = self.theta - lr * gr
        grad.close()
        e1 = self.prepare()
        rec = {"selected": a, "max_abs_pool_gradient": float(abs(g[a])), "energy_before": e0,
               "energy_after": e1, "descent": energies, "n_ops": len(self.ops)}
        self.history.append(rec)
        return rec


def bond_dimension_scan(n_qubits: int, gates, plan: "binding.PauliSum", bits, bonds, cutoff: float = 1e-14,
                        prec: str = "c128", stream: int | None = None) -> list[float]:
    """Energy of one circuit at every bond dimension in `bonds` (increasing)."""
    q0, q1, u = gates
    out = []
    for D in bonds:
        m = binding.Mps(n_qubits, int(D), cutoff, bits=bits, stream=stream)
        m.apply_gates(q0, q1, u)
        out.append(m.expect(plan, prec))
        m.close()
    return out


def select_bond_dimension(bonds, energies, tol: float = 1e-3):
    """First D_i with |E(D_i) - E(D_i+1)| < tol, or None."""
    for i in range(len(bonds) - 1):
        if abs(energies[i] - energies[i + 1]) < tol:
            return bonds[i]
    return None
