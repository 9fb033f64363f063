"""Reduced density matrices: the oracle's ladder-operator RDMs pinned by
closed forms and sum rules (Hartree-Fock determinant, particle number,
partial trace, the energy of the JW Hamiltonian), and the JW row expansion
used on the device checked against them on dense states."""

import math

import numpy as np

from oracle import dense_apply_gates, dense_energy, dense_expect_pauli, dense_product_state, \
    dense_rdm1, dense_rdm2
from workloads import hf_bits, jw_hamiltonian, random_integrals, uccsd_gates, workload_rng
from workloads.circuits import uccsd_n_params
from workloads.rdm import one_rdm_rows, two_rdm_rows


def _uccsd_state(n, ne, seed, scale=0.3):
    theta = workload_rng(seed, 1).uniform(-scale, scale, size=uccsd_n_params(n, ne))
    return dense_apply_gates(dense_product_state(hf_bits(n, ne)), uccsd_gates(n, ne, theta))


def test_hartree_fock_rdms_closed_form():
    n, ne = 6, 3
    psi = dense_product_state(hf_bits(n, ne))
    occ = np.array(hf_bits(n, ne), float)
    g1 = dense_rdm1(psi)
    assert np.allclose(g1, np.diag(occ), atol=1e-15)
    g2 = dense_rdm2(psi)
    d = np.eye(n)
    ref = np.einsum("p,q,ps,qr->pqrs", occ, occ, d, d) - np.einsum("p,q,pr,qs->pqrs", occ, occ, d, d)
    assert np.allclose(g2, ref, atol=1e-15)


def test_rdm_sum_rules_and_energy():
    n_s, ne = 3, 2
    n = 2 * n_s
    psi = _uccsd_state(n, ne, 61)
    g1 = dense_rdm1(psi)
    g2 = dense_rdm2(psi)
    assert abs(np.trace(g1) - ne) < 1e-12
    assert np.allclose(g1, g1.conj().T, atol=1e-13)
    assert np.allclose(np.einsum("pqqs->ps", g2), (ne - 1) * g1, atol=1e-12)
    assert np.allclose(g2, -g2.transpose(1, 0, 2, 3), atol=1e-13)
    # E = sum h_pq gamma + 1/2 sum (pq|rs) Gamma_{p s, r t, s' t, q s}: the
    # Hamiltonian's second-quantised form, against its JW Pauli sum
    h, g = random_integrals(n_s, workload_rng(61, 0))
    ps = jw_hamiltonian(h, g)
    e_pauli = dense_energy(psi, ps.codes, ps.coeffs)
    e = 0.0
    for p in range(n_s):
        for q in range(n_s):
            for s in range(2):
                e += h[p, q] * g1[2 * p + s, 2 * q + s].real
    for p in range(n_s):
        for q in range(n_s):
            for r in range(n_s):
                for s_ in range(n_s):
                    for a in range(2):
                        for b in range(2):
                            e += 0.5 * g[p, q, r, s_] * g2[2 * p + a, 2 * r + b, 2 * s_ + b, 2 * q + a].real
    assert abs(e - e_pauli) < 1e-11, (e, e_pauli)


def _apply_rows(rows, psi):
    per = np.array([dense_expect_pauli(psi, c).real for c in rows.strings.codes])
    out = np.array([math.fsum(rows.vals[a:b] * per[rows.cols[a:b]])
                    for a, b in zip(rows.row_ptr[:-1], rows.row_ptr[1:])])
    return out[0::2] + 1j * out[1::2]


def test_jw_rows_reproduce_ladder_rdms():
    n, ne = 6, 3
    rng = np.random.default_rng(4)
    psi = (rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)).reshape((2,) * n)
    psi /= np.linalg.norm(psi)
    r1 = one_rdm_rows(n)
    assert np.max(np.abs(_apply_rows(r1, psi).reshape(n, n) - dense_rdm1(psi))) < 1e-13
    r2 = two_rdm_rows(n)
    val = _apply_rows(r2, psi)
    g2 = dense_rdm2(psi)
    p, q, r, s = r2.elements.T
    assert np.max(np.abs(val - g2[p, q, r, s])) < 1e-13
