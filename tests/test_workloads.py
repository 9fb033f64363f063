"""Pins for the synthetic input generators (Hamiltonian, circuits)."""

import numpy as np
import pytest
import scipy.linalg

from workloads import (
    brickwork_gates, fuse_gates, generic_term_count, hf_bits, jw_hamiltonian,
    pauli_exponential_gates, random_integrals, uccsd_gates, workload_rng,
)
from workloads.circuits import uccsd_excitations, uccsd_n_params
from oracle import dense_apply_gates, dense_pauli_matrix, dense_product_state, dense_energy
from tests import fermion_ref as fr


@pytest.fixture(scope="module")
def small_h():
    h, g = random_integrals(3, workload_rng(99, 0))
    return h, g, jw_hamiltonian(h, g)


def test_integral_symmetry():
    h, g = random_integrals(4, workload_rng(1, 0))
    assert np.allclose(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (1, 0, 3, 2), (3, 2, 1, 0)]:
        assert np.array_equal(g, g.transpose(perm))
    # every orbit drawn once: number of distinct values = number of 8-fold orbits
    npair = 4 * 5 // 2
    assert np.unique(g).size == npair * (npair + 1) // 2


def test_jw_matches_fermionic_matrix(small_h):
    h, g, ps = small_h
    Hf = fr.hamiltonian_matrix(h, g)
    Hq = fr.pauli_sum_matrix(ps.codes, ps.coeffs)
    assert np.max(np.abs(Hf - Hq)) < 1e-12


def test_jw_matches_fermionic_matrix_8q():
    h, g = random_integrals(4, workload_rng(1, 0))
    ps = jw_hamiltonian(h, g)
    Hf = fr.hamiltonian_matrix(h, g)
    Hq = fr.pauli_sum_matrix(ps.codes, ps.coeffs)
    assert np.max(np.abs(Hf - Hq)) < 1e-12
    assert np.max(np.abs(Hq - Hq.conj().T)) < 1e-14
    N = fr.number_operator(8)
    Sz = fr.sz_operator(8)
    assert np.max(np.abs(Hq @ N - N @ Hq)) < 1e-12
    assert np.max(np.abs(Hq @ Sz - Sz @ Hq)) < 1e-12


@pytest.mark.parametrize("n_s", [2, 3, 4, 5, 6])
def test_term_count(n_s):
    h, g = random_integrals(n_s, workload_rng(7, 0))
    assert jw_hamiltonian(h, g).n_terms == generic_term_count(n_s)


def test_hf_energy_closed_form(small_h):
    h, g, ps = small_h
    psi = dense_product_state(hf_bits(6, 2))
    e = dense_energy(psi, ps.codes, ps.coeffs)
    assert abs(e - fr.hf_energy_closed_form(h, g, 2)) < 1e-12


@pytest.mark.parametrize("code", [
    [1, 0, 0], [2, 3, 1], [1, 0, 2], [3, 0, 0, 3], [2, 3, 0, 0, 1], [0, 1, 2, 0], [1, 1, 1, 1],
    [2, 0, 0, 0, 2],
])
def test_pauli_exponential_matches_expm(code):
    code = np.array(code, dtype=np.uint8)
    n = code.size
    phi = 0.3711
    gates = pauli_exponential_gates(code, phi)
    assert all(g.q1 < 0 or g.q1 == g.q0 + 1 for g in gates)
    U = np.zeros((1 << n, 1 << n), dtype=complex)
    for b in range(1 << n):
        e = np.zeros(1 << n, dtype=complex)
        e[b] = 1
        U[:, b] = dense_apply_gates(e.reshape((2,) * n), gates).reshape(-1)
    ref = scipy.linalg.expm(1j * phi * dense_pauli_matrix(code))
    assert np.max(np.abs(U - ref)) < 1e-13


def _tau_matrix(n, left, right):
    m = np.eye(1 << n)
    for o in left:
        m = m @ fr.ladder(n, o, True)
    for o in right:
        m = m @ fr.ladder(n, o, False)
    return m


@pytest.mark.parametrize("fuse", [False, True])
def test_uccsd_circuit_matches_trotter_product(fuse):
    n, ne = 6, 2
    theta = workload_rng(11, 1).uniform(-0.1, 0.1, size=uccsd_n_params(n, ne))
    gates = uccsd_gates(n, ne, theta)
    if fuse:
        gates = fuse_gates(gates, n)
    psi = dense_apply_gates(dense_product_state(hf_bits(n, ne)), gates).reshape(-1)
    singles, doubles = uccsd_excitations(n, ne)
    exc = [((a,), (i,)) for (i, a) in singles] + [((a, b), (i, j)) for (i, j, a, b) in doubles]
    ref = dense_product_state(hf_bits(n, ne)).reshape(-1)
    for t, (left, right) in zip(theta, exc):
        tau = _tau_matrix(n, left, right)
        ref = scipy.linalg.expm(t * (tau - tau.T)) @ ref
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_uccsd_counts():
    s, d = uccsd_excitations(8, 4)
    assert (len(s), len(d)) == (8, 18)
    s, d = uccsd_excitations(24, 12)
    assert (len(s), len(d)) == (72, 1746)


def test_brickwork_structure_and_fuse():
    n, L = 6, 3
    ang = workload_rng(3, 1).uniform(-np.pi, np.pi, size=(L, n, 2))
    gates = brickwork_gates(n, ang)
    assert sum(g.q1 >= 0 for g in gates) == L * (n - 1)
    fused = fuse_gates(gates, n)
    assert all(g.q1 >= 0 for g in fused)  # every rotation folds into an even CNOT
    psi0 = dense_product_state(hf_bits(n, 2))
    a = dense_apply_gates(psi0, gates)
    b = dense_apply_gates(psi0, fused)
    assert np.max(np.abs(a - b)) < 1e-13
