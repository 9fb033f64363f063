"""Pins for the FP64 oracle: each function is tied to something other than
itself (brute-force statevectors, LAPACK, closed forms, sum rules, the
variational bound), and planted mistakes are shown to be caught."""

import math

import numpy as np
import pytest

from oracle import (
    MpsOracle, dense_apply_gates, dense_apply_pauli, dense_energy, dense_expect_pauli,
    dense_pauli_matrix, dense_product_state, one_sided_jacobi_svd,
)
from oracle.jacobi import JacobiNoConvergence
from workloads import (
    brickwork_gates, build_config, fuse_gates, hf_bits, jw_hamiltonian, random_integrals,
    uccsd_gates, workload_rng,
)
from workloads.circuits import Gate, uccsd_n_params
from tests import fermion_ref as fr


def _rand_state(n, seed):
    r = np.random.default_rng(seed)
    v = r.normal(size=1 << n) + 1j * r.normal(size=1 << n)
    return (v / np.linalg.norm(v)).reshape((2,) * n)


def _all_codes(n):
    return np.array(np.meshgrid(*[range(4)] * n, indexing="ij")).reshape(n, -1).T.astype(np.uint8)


# ------------------------------------------------------------------ dense

def test_dense_pauli_action_matches_kron():
    n = 4
    psi = _rand_state(n, 1)
    for code in _all_codes(n)[::7]:
        a = dense_apply_pauli(psi, code).reshape(-1)
        b = dense_pauli_matrix(code) @ psi.reshape(-1)
        assert np.max(np.abs(a - b)) < 1e-14


def test_pure_state_sum_rule():
    """sum over all 4^N strings of <P>^2 = 2^N for a pure state."""
    n = 5
    psi = _rand_state(n, 2)
    tot = math.fsum(abs(dense_expect_pauli(psi, c)) ** 2 for c in _all_codes(n))
    assert abs(tot - 2 ** n) < 1e-10


def test_ghz_closed_forms():
    n = 5
    psi = np.zeros((2,) * n, dtype=complex)
    psi[(0,) * n] = psi[(1,) * n] = 1 / math.sqrt(2)
    assert abs(dense_expect_pauli(psi, np.array([1] * n)) - 1) < 1e-14
    assert abs(dense_expect_pauli(psi, np.array([3, 3, 0, 0, 0])) - 1) < 1e-14
    assert abs(dense_expect_pauli(psi, np.array([3, 0, 0, 0, 0]))) < 1e-14
    # Y^{x2} X^{x3}: <GHZ| Y Y X X X |GHZ> = i^2 = -1
    assert abs(dense_expect_pauli(psi, np.array([2, 2, 1, 1, 1])) + 1) < 1e-14


# ------------------------------------------------------------------ Jacobi SVD

@pytest.mark.parametrize("shape", [(6, 6), (12, 8), (16, 16), (9, 5), (5, 9)])
def test_jacobi_matches_lapack(shape):
    r = np.random.default_rng(sum(shape))
    A = r.normal(size=shape) + 1j * r.normal(size=shape)
    U, s, V = one_sided_jacobi_svd(A)
    s_ref = np.linalg.svd(A, compute_uv=False)
    k = min(shape)
    assert np.max(np.abs(s[:k] - s_ref) / s_ref[0]) < 1e-13
    if s.size > k:
        assert np.max(np.abs(s[k:])) < 1e-13 * s_ref[0]
    assert np.max(np.abs(A @ V - U * s)) < 1e-13 * s_ref[0]
    assert np.max(np.abs(V.conj().T @ V - np.eye(shape[1]))) < 1e-13
    Uk = U[:, :k]
    assert np.max(np.abs(Uk.conj().T @ Uk - np.eye(k))) < 1e-13


def test_jacobi_known_spectrum():
    r = np.random.default_rng(5)
    n = 10
    Q, _ = np.linalg.qr(r.normal(size=(n, n)) + 1j * r.normal(size=(n, n)))
    P, _ = np.linalg.qr(r.normal(size=(n, n)) + 1j * r.normal(size=(n, n)))
    sig = np.array([3.0, 2.0, 1.5, 1.0, 0.5, 1e-3, 1e-6, 1e-9, 0.0, 0.0])
    A = Q @ np.diag(sig) @ P.conj().T
    _, s, _ = one_sided_jacobi_svd(A)
    assert np.max(np.abs(s - sig)) < 1e-14 * 3


def test_jacobi_rotation_orthogonalises_pair():
    """The complex rotation makes a_i'^+ a_j' vanish (reading of tau/t/c/s)."""
    r = np.random.default_rng(8)
    A = r.normal(size=(7, 2)) + 1j * r.normal(size=(7, 2))
    U, s, V = one_sided_jacobi_svd(A)
    B = A @ V
    assert abs(np.vdot(B[:, 0], B[:, 1])) < 1e-14 * np.linalg.norm(A) ** 2


def test_jacobi_sweep_limit_raises():
    r = np.random.default_rng(9)
    A = r.normal(size=(12, 12)) + 1j * r.normal(size=(12, 12))
    with pytest.raises(JacobiNoConvergence):
        one_sided_jacobi_svd(A, max_sweeps=1)


# ------------------------------------------------------------------ MPS

def test_mps_product_state_expectations():
    bits = [1, 0, 1, 1, 0]
    m = MpsOracle(5, 4, bits=bits)
    for q in range(5):
        code = np.zeros(5, dtype=np.uint8)
        code[q] = 3
        assert abs(m.expect_pauli(code) - (1 - 2 * bits[q])) < 1e-15
        code[q] = 1
        assert abs(m.expect_pauli(code)) < 1e-15


def test_mps_c1_matches_statevector():
    w = build_config(1)
    psi = dense_apply_gates(dense_product_state(w.bits), w.gates)
    m = MpsOracle(w.n_qubits, 16, 1e-14, w.bits)
    m.apply_gates(w.gates)
    assert np.max(np.abs(m.to_statevector() - psi)) < 1e-12
    assert m.discarded < 1e-25
    m.canonicalize()
    assert abs(m.norm_before_canon - 1) < 1e-13
    assert m.right_canonical_residual() < 1e-13
    e_mps = m.energy(w.psum.codes, w.psum.coeffs)
    e_dense = dense_energy(psi, w.psum.codes, w.psum.coeffs)
    assert abs(e_mps - e_dense) < 1e-12
    per = m.expect_terms(w.psum.codes)
    assert np.max(np.abs(per.imag)) < 1e-13


@pytest.mark.parametrize("n,layers,seed", [(6, 4, 0), (9, 3, 1), (10, 5, 2)])
def test_mps_brickwork_untruncated_matches_statevector(n, layers, seed):
    ang = np.random.default_rng(seed).uniform(-np.pi, np.pi, size=(layers, n, 2))
    gates = brickwork_gates(n, ang)
    bits = hf_bits(n, n // 2)
    psi = dense_apply_gates(dense_product_state(bits), gates)
    m = MpsOracle(n, 64, 1e-14, bits)
    m.apply_gates(gates)
    ph = m.to_statevector()
    assert np.max(np.abs(ph - psi)) < 1e-12
    m.canonicalize()
    assert m.right_canonical_residual() < 1e-13
    code = np.array([1, 3, 3, 2] + [0] * (n - 6) + [2, 1], dtype=np.uint8)
    assert abs(m.expect_pauli(code) - dense_expect_pauli(psi, code)) < 1e-12


def test_hastings_identity_without_truncation():
    """Without truncation B~_q = U lam~ / lam_q (Eq. Uλ/λ) and B~_{q+1} is right-canonical."""
    n = 6
    ang = np.random.default_rng(3).uniform(-np.pi, np.pi, size=(2, n, 2))
    m = MpsOracle(n, 64, 1e-14, hf_bits(n, 3))
    m.apply_gates(brickwork_gates(n, ang))
    m.canonicalize()
    q = 2
    u = np.kron(np.array([[0.6, 0.8j], [0.8j, 0.6]]), np.eye(2)) @ \
        np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    lam_l = m.lam[q].copy()
    Bl, Br = m.B[q], m.B[q + 1]
    dl, dr = Bl.shape[1], Br.shape[2]
    theta = np.einsum("alm,bmr->ablr", Bl, Br)
    C = np.einsum("cdab,ablr->cdlr", u.reshape(2, 2, 2, 2), theta).transpose(0, 2, 1, 3)
    Ct = np.tile(lam_l, 2)[:, None] * C.reshape(2 * dl, 2 * dr)
    U, s, _ = np.linalg.svd(Ct, full_matrices=False)
    m.apply_2q(q, u)
    k = m.lam[q + 1].size
    ref = (U[:, :k] * s[:k]) / np.tile(lam_l, 2)[:, None]  # U lam~ / lam_q
    got = m.B[q].reshape(2 * dl, k)
    # equal up to the per-column phase freedom of the SVD
    ph = np.sum(got.conj() * ref, axis=0)
    ph = ph / np.abs(ph)
    assert np.max(np.abs(got * ph[None, :] - ref / np.linalg.norm(s[:k]))) < 1e-12
    g = np.einsum("sab,scb->ac", m.B[q + 1], m.B[q + 1].conj())
    assert np.max(np.abs(g - np.eye(k))) < 1e-13


def test_truncated_mps_transfer_equals_full_contraction():
    n, layers = 10, 6
    ang = np.random.default_rng(4).uniform(-np.pi, np.pi, size=(layers, n, 2))
    m = MpsOracle(n, 6, 1e-14, hf_bits(n, 5))
    m.apply_gates(fuse_gates(brickwork_gates(n, ang), n))
    assert m.discarded > 1e-6  # truncation really happened
    m.canonicalize()
    psi = m.to_statevector()
    r = np.random.default_rng(6)
    for _ in range(20):
        code = r.integers(0, 4, size=n).astype(np.uint8)
        a = m.expect_pauli(code)
        b = m.expect_pauli_full(code)
        c = dense_expect_pauli(psi, code) / np.vdot(psi, psi)
        assert abs(a - b) < 1e-12 and abs(a - c) < 1e-12


def test_canonicalize_idempotent_and_normalising():
    n = 8
    ang = np.random.default_rng(7).uniform(-np.pi, np.pi, size=(4, n, 2))
    m = MpsOracle(n, 4, 1e-14, hf_bits(n, 4))
    m.apply_gates(brickwork_gates(n, ang))
    m.canonicalize()
    lam1 = [l.copy() for l in m.lam]
    m.canonicalize()
    assert abs(m.norm_before_canon - 1) < 1e-13
    for a, b in zip(lam1, m.lam):
        assert np.max(np.abs(a - b)) < 1e-13
    # lam are Schmidt values: compare with the SVD of the dense state
    psi = m.to_statevector().reshape(1 << 3, -1)
    s = np.linalg.svd(psi, compute_uv=False)
    k = m.lam[3].size
    assert np.max(np.abs(s[:k] - m.lam[3])) < 1e-12


def test_variational_bound_and_number_conservation():
    n_s, ne = 4, 4
    h, g = random_integrals(n_s, workload_rng(21, 0))
    ps = jw_hamiltonian(h, g)
    Hq = fr.pauli_sum_matrix(ps.codes, ps.coeffs)
    e0 = float(np.linalg.eigvalsh(Hq)[0])
    theta = workload_rng(21, 1).uniform(-0.5, 0.5, size=uccsd_n_params(8, ne))
    for D, cut in [(16, 1e-14), (3, 1e-14)]:
        m = MpsOracle(8, D, cut, hf_bits(8, ne))
        m.apply_gates(uccsd_gates(8, ne, theta))
        e = m.energy(ps.codes, ps.coeffs)
        assert e >= e0 - 1e-10
    # number of electrons conserved by UCCSD without truncation
    m = MpsOracle(8, 16, 1e-14, hf_bits(8, ne))
    m.apply_gates(uccsd_gates(8, ne, theta))
    m.canonicalize()
    nocc = 0.0
    for j in range(8):
        code = np.zeros(8, dtype=np.uint8)
        code[j] = 3
        nocc += 0.5 * (1 - m.expect_pauli(code).real)
    assert abs(nocc - ne) < 1e-10


def test_hf_energy_through_mps():
    n_s, ne = 4, 4
    h, g = random_integrals(n_s, workload_rng(22, 0))
    ps = jw_hamiltonian(h, g)
    m = MpsOracle(8, 16, 1e-14, hf_bits(8, ne))
    m.apply_gates(uccsd_gates(8, ne, np.zeros(uccsd_n_params(8, ne))))
    e = m.energy(ps.codes, ps.coeffs)
    assert abs(e - fr.hf_energy_closed_form(h, g, ne)) < 1e-12


def test_jacobi_svd_mps_equals_lapack_mps():
    n = 7
    ang = np.random.default_rng(8).uniform(-np.pi, np.pi, size=(3, n, 2))
    gates = fuse_gates(brickwork_gates(n, ang), n)
    a = MpsOracle(n, 5, 1e-14, hf_bits(n, 3))
    b = MpsOracle(n, 5, 1e-14, hf_bits(n, 3), svd="jacobi")
    a.apply_gates(gates)
    b.apply_gates(gates)
    a.canonicalize()
    b.canonicalize()
    r = np.random.default_rng(9)
    for _ in range(10):
        code = r.integers(0, 4, size=n).astype(np.uint8)
        assert abs(a.expect_pauli(code) - b.expect_pauli(code)) < 1e-12


# ------------------------------------------------------------------ planted mistakes

def _c1_error(monkeypatch_fn):
    w = build_config(1)
    psi = dense_apply_gates(dense_product_state(w.bits), w.gates)
    m = MpsOracle(w.n_qubits, 16, 1e-14, w.bits)
    monkeypatch_fn(m)
    m.apply_gates(w.gates)
    e = m.energy(w.psum.codes, w.psum.coeffs)
    return abs(e - dense_energy(psi, w.psum.codes, w.psum.coeffs))


def test_planted_transposed_operand_is_caught():
    def plant(m):
        orig = m._transfer

        def bad(L, q, c):
            B = m.B[q]
            from oracle.mps import _PAULI
            sig = _PAULI[c]
            out = np.zeros((B.shape[2], B.shape[2]), dtype=complex)
            for s in range(2):
                for sp in range(2):
                    if sig[s, sp] != 0:
                        out += sig[s, sp] * (B[s].T @ L @ B[sp])  # missing conjugate
            return out
        m._transfer = bad
    assert _c1_error(plant) > 1e-6


def _single_gate_truncation_error(plant=None):
    """Apply one truncating gate to an exact canonical MPS and compare with the
    Eckart-Young optimum of the dense state cut at the same bond."""
    n, q, k = 8, 3, 3
    ang = np.random.default_rng(12).uniform(-np.pi, np.pi, size=(3, n, 2))
    m = MpsOracle(n, 64, 1e-14, hf_bits(n, 4))
    m.apply_gates(brickwork_gates(n, ang))
    m.canonicalize()
    psi = m.to_statevector()
    u = np.kron(np.array([[0.6, 0.8j], [0.8j, 0.6]]), np.array([[0.8, -0.6], [0.6, 0.8]])) @ \
        np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    ex = dense_apply_gates(psi, [Gate(q, q + 1, u)]).reshape(1 << (q + 1), -1)
    U, s, Vh = np.linalg.svd(ex, full_matrices=False)
    opt = (U[:, :k] * s[:k]) @ Vh[:k]
    opt = opt / np.linalg.norm(opt)
    m.max_bond = k
    if plant is not None:
        plant(m)
    m.apply_2q(q, u)
    got = m.to_statevector().reshape(opt.shape)
    return abs(1 - abs(np.vdot(opt, got)))


def test_single_gate_truncation_is_optimal():
    assert _single_gate_truncation_error() < 1e-12


def test_planted_lambda_scaling_mistake_is_caught():
    def plant(m):
        orig = m.apply_2q

        def bad(q, u):
            m.lam[q] = np.sqrt(m.lam[q])  # wrong power of lambda in Eq. (C~)
            orig(q, u)
        m.apply_2q = bad
    assert _single_gate_truncation_error(plant) > 1e-6


def test_planted_sign_mistake_in_pauli_is_caught():
    """A real Hamiltonian has an even number of Y per string, so a flipped Y
    is invisible in the energy; per-string expectations against the dense
    statevector catch it."""
    from oracle import mps as mps_mod
    n = 6
    ang = np.random.default_rng(13).uniform(-np.pi, np.pi, size=(3, n, 2))
    gates = brickwork_gates(n, ang)
    psi = dense_apply_gates(dense_product_state(hf_bits(n, 3)), gates)
    m = MpsOracle(n, 64, 1e-14, hf_bits(n, 3))
    m.apply_gates(gates)
    m.canonicalize()
    code = np.array([0, 2, 3, 1, 0, 0], dtype=np.uint8)  # one Y
    ref = dense_expect_pauli(psi, code)
    assert abs(m.expect_pauli(code) - ref) < 1e-12
    assert abs(ref) > 1e-3
    saved = mps_mod._PAULI[2].copy()
    try:
        mps_mod._PAULI[2] = saved.conj()  # Y with the wrong sign
        assert abs(m.expect_pauli(code) - ref) > 1e-6
    finally:
        mps_mod._PAULI[2] = saved
