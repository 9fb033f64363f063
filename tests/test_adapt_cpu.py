"""Windowed qubit-ADAPT pool and selection rule: the pool against an
independent construction from the excitation structure, the parameter-shift
pool derivative against the commutator formula on dense states, and one
ADAPT iteration of the module on dense stand-in handles."""

import math
import types

import numpy as np

from oracle import dense_apply_gates, dense_apply_pauli, dense_energy, dense_product_state
from workloads import hf_bits, jw_hamiltonian, random_integrals, workload_rng
from workloads.circuits import pauli_exponential_gates, qubit_adapt_pool

X, Y = 1, 2


def _independent_pool(n, window):
    """XY / YX on every spin-conserving orbital pair, and the eight odd-Y
    X/Y patterns on every four orbitals that carry a spin-conserving double,
    inside a window of `window` spatial orbitals."""
    out = set()
    ok = lambda *o: max(x // 2 for x in o) - min(x // 2 for x in o) < window  # noqa: E731
    for p in range(n):
        for q in range(p):
            if p % 2 == q % 2 and ok(p, q):
                for a, b in ((X, Y), (Y, X)):
                    c = [0] * n
                    c[p], c[q] = a, b
                    out.add(tuple(c))
    for quad in __import__("itertools").combinations(range(n), 4):
        if not ok(*quad):
            continue
        spins = sorted(o % 2 for o in quad)
        if spins not in ([0, 0, 1, 1], [0, 0, 0, 0], [1, 1, 1, 1]):
            continue
        for pat in __import__("itertools").product((X, Y), repeat=4):
            if sum(1 for x in pat if x == Y) % 2 == 1:
                c = [0] * n
                for o, v in zip(quad, pat):
                    c[o] = v
                out.add(tuple(c))
    return out


def test_pool_matches_independent_construction():
    for n, w in ((8, 5), (12, 3), (12, 5)):
        pool = qubit_adapt_pool(n, w)
        got = {tuple(int(x) for x in row) for row in pool}
        assert len(got) == pool.shape[0]
        assert got == _independent_pool(n, w), (n, w)
        assert not np.any(pool == 3)
        assert np.all(np.sum(pool == Y, axis=1) % 2 == 1)


def test_shift_derivative_equals_commutator():
    n_s, n = 3, 6
    h, g = random_integrals(n_s, workload_rng(71, 0))
    ps = jw_hamiltonian(h, g)
    rng = np.random.default_rng(1)
    psi = (rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)).reshape((2,) * n)
    psi /= np.linalg.norm(psi)
    hpsi = sum(c * dense_apply_pauli(psi, code) for code, c in zip(ps.codes, ps.coeffs))
    for P in qubit_adapt_pool(n, 3)[:25]:
        plus = dense_energy(dense_apply_gates(psi, pauli_exponential_gates(P, math.pi / 4)), ps.codes, ps.coeffs)
        minus = dense_energy(dense_apply_gates(psi, pauli_exponential_gates(P, -math.pi / 4)), ps.codes, ps.coeffs)
        comm = -2.0 * np.vdot(hpsi.ravel(), dense_apply_pauli(psi, P).ravel()).imag
        assert abs((plus - minus) - comm) < 1e-12


def test_adapt_iteration_on_dense_handles(monkeypatch):
    from paper_2303_03681_amd import adapt, gradients
    from tests.test_gradients_cpu import _fake_binding
    fake = _fake_binding()
    monkeypatch.setattr(adapt, "binding", fake)
    monkeypatch.setattr(gradients, "binding", fake)
    n_s, n = 3, 6
    h, g = random_integrals(n_s, workload_rng(72, 0))
    ps = jw_hamiltonian(h, g)
    plan = types.SimpleNamespace(codes=ps.codes, coeffs=ps.coeffs)
    pool = qubit_adapt_pool(n, 3)
    bits = hf_bits(n, 2)
    ad = adapt.QubitAdapt(n, plan, pool, 8, bits=bits, batch=7)
    psi = dense_product_state(bits)
    hpsi = sum(c * dense_apply_pauli(psi, code) for code, c in zip(ps.codes, ps.coeffs))
    comm = np.array([-2.0 * np.vdot(hpsi.ravel(), dense_apply_pauli(psi, P).ravel()).imag for P in pool])
    ad.prepare()
    assert np.max(np.abs(ad.pool_gradients() - comm)) < 1e-12
    rec = ad.iterate(opt_steps=4, lr=0.2)
    # ties between symmetric pool strings are common: the choice must reach the maximum
    assert abs(abs(comm[rec["selected"]]) - np.max(np.abs(comm))) < 1e-12
    assert rec["energy_after"] < rec["energy_before"]
