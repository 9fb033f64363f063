"""Parameter-shift gradients: the shift rule and the chain rule over the
Pauli exponentials of UCCSD, pinned on dense statevectors (oracle) against
central finite differences; then the gradient module's prefix caching and
batching run on the CPU with a dense stand-in for the device handles."""

import math
import types

import numpy as np
import pytest

from oracle import dense_apply_gate, dense_apply_gates, dense_energy, dense_pauli_matrix, \
    dense_product_state
from workloads import hf_bits, jw_hamiltonian, random_integrals, workload_rng
from workloads.circuits import pauli_exponential_gates, uccsd_exponentials, uccsd_gates


def _dense_energy(n, ne, theta, ps):
    psi = dense_apply_gates(dense_product_state(hf_bits(n, ne)), uccsd_gates(n, ne, theta))
    return dense_energy(psi, ps.codes, ps.coeffs)


def _hamiltonian(n_s, seed):
    h, g = random_integrals(n_s, workload_rng(seed, 0))
    return jw_hamiltonian(h, g)


def test_shift_rule_single_exponential():
    """E(phi + pi/4) - E(phi - pi/4) = dE/dphi for exp(i phi P), P^2 = 1."""
    rng = np.random.default_rng(0)
    n = 4
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 = (psi0 / np.linalg.norm(psi0)).reshape((2,) * n)
    codes = rng.integers(0, 4, size=(12, n)).astype(np.uint8)
    coeffs = rng.normal(size=12)
    P = np.array([2, 0, 1, 3], np.uint8)

    def E(phi):
        return dense_energy(dense_apply_gates(psi0, pauli_exponential_gates(P, phi)), codes, coeffs)
    for phi in (0.0, 0.37, -1.2):
        shift = E(phi + math.pi / 4) - E(phi - math.pi / 4)
        h = 1e-5
        fd = (E(phi + h) - E(phi - h)) / (2 * h)
        assert abs(shift - fd) < 1e-8, (phi, shift, fd)
    # the compiled gates are exp(i phi P) itself
    cols = []
    for c in range(1 << n):
        e = np.zeros(1 << n, dtype=complex)
        e[c] = 1.0
        cols.append(dense_apply_gates(e.reshape((2,) * n), pauli_exponential_gates(P, 0.3)).ravel())
    U = np.stack(cols, axis=1)
    ref = math.cos(0.3) * np.eye(1 << n) + 1j * math.sin(0.3) * dense_pauli_matrix(P)
    assert np.max(np.abs(U - ref)) < 1e-12


def test_uccsd_chain_rule_matches_finite_differences():
    n, ne = 6, 2
    ps = _hamiltonian(n // 2, 51)
    exps = uccsd_exponentials(n, ne)
    n_par = 1 + max(j for j, _, _ in exps)
    theta = workload_rng(51, 1).uniform(-0.2, 0.2, size=n_par)
    psi_hf = dense_product_state(hf_bits(n, ne))
    grad = np.zeros(n_par)
    for k, (j, code, c) in enumerate(exps):
        e = []
        for s in (1, -1):
            psi = psi_hf
            for kk, (jj, cc_code, cc) in enumerate(exps):
                phi = theta[jj] * cc + (s * math.pi / 4 if kk == k else 0.0)
                psi = dense_apply_gates(psi, pauli_exponential_gates(cc_code, phi))
            e.append(dense_energy(psi, ps.codes, ps.coeffs))
        grad[j] += c * (e[0] - e[1])
    h = 1e-5
    for j in range(n_par):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (_dense_energy(n, ne, tp, ps) - _dense_energy(n, ne, tm, ps)) / (2 * h)
        assert abs(grad[j] - fd) < 1e-8, (j, grad[j], fd)


class _DenseMps:
    """Dense statevector with the handle methods the gradient module uses."""

    def __init__(self, n_qubits, max_bond, cutoff, bits=None, stream=None):
        self.n = n_qubits
        self.psi = dense_product_state(bits if bits is not None else [0] * n_qubits)

    def reset(self, bits=None):
        self.psi = dense_product_state(bits if bits is not None else [0] * self.n)

    def copy_from(self, src):
        self.psi = src.psi.copy()

    def apply_gates(self, q0, q1, u):
        u = np.asarray(u).reshape(len(q0), 16, 2)
        for a, b, m in zip(q0, q1, u):
            z = m[:, 0] + 1j * m[:, 1]
            self.psi = dense_apply_gate(self.psi, int(a), int(b), z[:16].reshape(4, 4) if b >= 0
                                        else z[:4].reshape(2, 2))

    def expect(self, plan, prec):
        return dense_energy(self.psi, plan.codes, plan.coeffs) / np.vdot(self.psi.ravel(), self.psi.ravel()).real

    def close(self):
        pass


def _fake_binding():
    class MpsError(RuntimeError):
        pass

    def apply_gates_multi(handles, lists):
        for h, l in zip(handles, lists):
            h.apply_gates(*l)
        return np.array([len(l[0]) for l in lists])

    def expect_multi(handles, plans, prec):
        return np.array([h.expect(p, prec) for h, p in zip(handles, plans)])
    return types.SimpleNamespace(Mps=_DenseMps, MpsError=MpsError, apply_gates_multi=apply_gates_multi,
                                 expect_multi=expect_multi)


@pytest.mark.parametrize("batch", [1, 3])
def test_gradient_module_prefix_caching_on_dense_handles(monkeypatch, batch):
    from paper_2303_03681_amd import gradients
    monkeypatch.setattr(gradients, "binding", _fake_binding())
    n, ne = 6, 2
    ps = _hamiltonian(n // 2, 52)
    plan = types.SimpleNamespace(codes=ps.codes, coeffs=ps.coeffs)
    gr = gradients.UccsdGradient(n, ne, plan, 8, bits=hf_bits(n, ne), batch=batch)
    theta = workload_rng(52, 1).uniform(-0.2, 0.2, size=gr.n_params)
    e, g = gr.energy_and_gradient(theta)
    assert abs(e - _dense_energy(n, ne, theta, ps)) < 1e-12
    h = 1e-5
    for j in range(gr.n_params):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (_dense_energy(n, ne, tp, ps) - _dense_energy(n, ne, tm, ps)) / (2 * h)
        assert abs(g[j] - fd) < 1e-8, (j, g[j], fd)
    assert gr.evaluations == 2 * len(gr.exps) + 1
    th, energies = gradients.gradient_descent(gr, theta, steps=3, lr=0.05)
    assert all(b < a for a, b in zip(energies, energies[1:]))
