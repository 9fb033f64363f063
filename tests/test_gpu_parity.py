"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
identical seeded inputs.  Tolerances: c128 energies within 1e-9 of the
oracle (absolute, Hartree), per-string values within 1e-10; c64 energies
within 1e-6 (FP32 rounding, about 6e-8 relative per product, accumulated
over chains of up to a few dozen transfer products); singular values within
1e-12 relative to the largest."""

import math

import numpy as np
import pytest

from oracle import MpsOracle, dense_apply_gates, dense_energy, dense_expect_pauli, \
    dense_product_state
from workloads import brickwork_gates, build_config, fuse_gates, hf_bits, jw_hamiltonian, \
    pack_gates, random_integrals, workload_rng
from workloads.circuits import Gate, gate_cnot

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _mps_state_from_gpu(m, n):
    """Contract the exported site tensors into a statevector (test-side numpy)."""
    psi = np.ones((1, 1), dtype=complex)
    for q in range(n):
        B, _ = m.export_site(q)
        psi = np.einsum("pa,sab->psb", psi, B).reshape(-1, B.shape[2])
    return psi.reshape((2,) * n)


def _apply(m, gates):
    q0, q1, u = pack_gates(gates)
    assert m.apply_gates(q0, q1, u) == len(gates)


def test_mfma_layout(gpu_lib):
    from paper_2303_03681_amd import binding
    out = binding.selftest_mfma()
    r = np.arange(16)[:, None]
    k = np.arange(4)[None, :]
    A = 1.0 + r + 0.5 * k
    B = 1.0 + 0.25 * np.arange(4)[:, None] - 0.125 * np.arange(16)[None, :]
    assert np.max(np.abs(out[0] - A @ B)) < 1e-12
    assert np.max(np.abs(out[1] - A @ B)) < 1e-4
    # 16x16x32 (bf16, f16): small integers, exact in 16 bits and in the FP32 sums
    i = np.arange(16)[:, None]
    kk = np.arange(32)[None, :]
    A32 = ((i + 2 * kk) % 7 - 3).astype(float)
    B32 = ((3 * np.arange(32)[:, None] + np.arange(16)[None, :]) % 5 - 2).astype(float)
    assert np.array_equal(out[2], A32 @ B32)
    assert np.array_equal(out[3], A32 @ B32)


@pytest.mark.parametrize("n,m", [(4, 6), (16, 16), (33, 20), (64, 64), (20, 300), (96, 512),
                                 (200, 64), (512, 512), (40, 700), (18, 18), (1024, 1024),
                                 (300, 1000), (1000, 520), (1023, 1022)])
def test_jacobi_svd_matches_lapack(gpu_lib, n, m):
    from paper_2303_03681_amd import binding
    _say(f"jacobi n={n} m={m}")
    r = np.random.default_rng(n * 1000 + m)
    A = r.normal(size=(n, m)) + 1j * r.normal(size=(n, m))
    sig, W, sweeps = binding.jacobi_svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    k = min(n, m)
    assert np.max(np.abs(sig[:k] - ref)) < 1e-12 * ref[0]
    assert np.all(sig[k:] < 1e-12 * ref[0])
    Wk = W[:k]
    assert np.max(np.abs(Wk @ Wk.conj().T - np.eye(k))) < 1e-12
    # every row of A lies in the span of the kept right singular vectors
    assert np.max(np.abs(A - (A @ Wk.conj().T) @ Wk)) < 1e-11 * ref[0]
    assert 1 <= sweeps <= 30


def test_c1_uccsd_end_to_end_vs_statevector(gpu_lib):
    from paper_2303_03681_amd import binding
    w = build_config(1)
    _say(f"C1: {len(w.gates)} gates, {w.psum.n_terms} strings")
    psi = dense_apply_gates(dense_product_state(w.bits), w.gates)
    e_ref = dense_energy(psi, w.psum.codes, w.psum.coeffs)
    m = binding.Mps(w.n_qubits, 16, 1e-14, bits=w.bits)
    _apply(m, w.gates)
    assert np.max(np.abs(_mps_state_from_gpu(m, w.n_qubits) - psi)) < 1e-11
    ps = binding.PauliSum(w.psum.codes, w.psum.coeffs)
    e, per = m.expect(ps, "c128", per_term=True)
    assert abs(e - e_ref) < 1e-10
    per_ref = np.array([dense_expect_pauli(psi, c).real for c in w.psum.codes])
    assert np.max(np.abs(per - per_ref)) < 1e-11
    assert abs(m.norm() - 1) < 1e-12
    assert list(m.bond_dims()) == [1, 2, 4, 8, 16, 8, 4, 2, 1]
    e64 = m.expect(ps, "c64")
    assert abs(e64 - e_ref) < 1e-5


def test_c1_canonicalize_preserves_state(gpu_lib):
    from paper_2303_03681_amd import binding
    w = build_config(1)
    psi = dense_apply_gates(dense_product_state(w.bits), w.gates)
    m = binding.Mps(w.n_qubits, 16, 1e-14, bits=w.bits)
    _apply(m, w.gates)
    m.canonicalize()
    phi = _mps_state_from_gpu(m, w.n_qubits)
    ov = np.vdot(phi, psi)
    assert abs(abs(ov) - 1) < 1e-11, ov
    assert np.max(np.abs(phi * (ov / abs(ov)) - psi)) < 1e-11
    for q in range(w.n_qubits):
        B, lam = m.export_site(q)
        g = np.einsum("sab,scb->ac", B, B.conj())
        assert np.max(np.abs(g - np.eye(g.shape[0]))) < 1e-12, q
        s = np.linalg.svd(psi.reshape(1 << q, -1), compute_uv=False)[:lam.size]
        assert np.max(np.abs(s - lam)) < 1e-12, q


def test_c1_unfused_gates_exercise_one_qubit_kernel(gpu_lib):
    from paper_2303_03681_amd import binding
    w = build_config(1, fuse=False)
    assert any(g.q1 < 0 for g in w.gates)
    psi = dense_apply_gates(dense_product_state(w.bits), w.gates)
    m = binding.Mps(w.n_qubits, 16, 1e-14, bits=w.bits)
    _apply(m, w.gates)
    assert np.max(np.abs(_mps_state_from_gpu(m, w.n_qubits) - psi)) < 1e-11


@pytest.mark.parametrize("n_s,layers,D", [(5, 6, 8), (6, 5, 12), (7, 4, 32)])
def test_truncated_brickwork_vs_oracle(gpu_lib, n_s, layers, D):
    from paper_2303_03681_amd import binding
    n = 2 * n_s
    _say(f"brickwork n={n} layers={layers} D={D}")
    h, g = random_integrals(n_s, workload_rng(60 + n_s, 0))
    ps = jw_hamiltonian(h, g)
    ang = workload_rng(60 + n_s, 1).uniform(-np.pi, np.pi, size=(layers, n, 2))
    gates = fuse_gates(brickwork_gates(n, ang), n)
    bits = hf_bits(n, n_s)
    o = MpsOracle(n, D, 1e-14, bits)
    o.apply_gates(gates)
    m = binding.Mps(n, D, 1e-14, bits=bits)
    _apply(m, gates)
    assert list(m.bond_dims()) == o.bond_dims()
    assert abs(m.discarded_weight() - o.discarded) < 1e-10 * max(1.0, o.discarded)
    o.canonicalize()
    plan = binding.PauliSum(ps.codes, ps.coeffs)
    e, per = m.expect(plan, "c128", per_term=True)
    ref = o.expect_terms(ps.codes).real
    assert np.max(np.abs(per - ref)) < 1e-10
    assert abs(e - math.fsum(ps.coeffs * ref)) < 1e-9
    assert abs(m.norm() - o.norm_before_canon) < 1e-10
    e64 = m.expect(plan, "c64")
    assert abs(e64 - e) < 1e-5
    for pr in ("split_bf16", "split_f16"):
        es, ps = m.expect(plan, pr, per_term=True)
        _say(f"  {pr}: |dE| {abs(es - e):.2e}, max |d<P>| {np.max(np.abs(ps - per)):.2e}")
        # bf16 split keeps ~16 significant bits per operand, f16 split ~22
        # (FP32 accumulation): measured |dE| <= 1.1e-6 and <= 2.4e-8 here
        assert abs(es - e) < (1e-5 if pr == "split_bf16" else 2e-7)
        assert np.max(np.abs(ps - per)) < (5e-5 if pr == "split_bf16" else 1e-6)


def _canonical_random_oracle(n, D, seed, layers=None):
    """A canonical oracle MPS with saturated bonds from a brickwork circuit."""
    ang = np.random.default_rng(seed).uniform(-np.pi, np.pi, size=(layers or n, n, 2))
    o = MpsOracle(n, D, 1e-14, hf_bits(n, n // 2))
    o.apply_gates(fuse_gates(brickwork_gates(n, ang), n))
    o.canonicalize()
    return o


def test_imported_state_expectations(gpu_lib):
    from paper_2303_03681_amd import binding
    n, D = 12, 24
    o = _canonical_random_oracle(n, D, 5, layers=6)
    m = binding.Mps(n, D, 1e-14)
    for q in range(n):
        m.import_site(q, o.B[q], o.lam[q])
    r = np.random.default_rng(7)
    codes = r.integers(0, 4, size=(300, n)).astype(np.uint8)
    codes[::7] = 0
    codes[1::7, :n - 2] = 0
    coeffs = r.normal(size=300)
    plan = binding.PauliSum(codes, coeffs)
    e, per = m.expect(plan, "c128", per_term=True)
    ref = o.expect_terms(codes).real
    assert np.max(np.abs(per - ref)) < 1e-11
    assert abs(e - math.fsum(coeffs * ref)) < 1e-10


def test_edge_cases(gpu_lib):
    from paper_2303_03681_amd import binding
    # one qubit
    m = binding.Mps(1, 4, 1e-14, bits=[1])
    plan = binding.PauliSum(np.array([[3], [0], [1]], np.uint8), np.array([2.0, 0.5, 1.0]))
    e, per = m.expect(plan, "c128", per_term=True)
    assert np.allclose(per, [-1.0, 1.0, 0.0], atol=1e-14) and abs(e - (-1.5)) < 1e-14
    m.apply_gate(0, -1, np.array([[0, 1], [1, 0]]))
    assert abs(m.expect(plan, "c128") - 2.5) < 1e-14
    # empty sum and identity-only sum
    m2 = binding.Mps(6, 4, 1e-14)
    assert m2.expect(binding.PauliSum(np.zeros((0, 6), np.uint8), np.zeros(0))) == 0.0
    assert abs(m2.expect(binding.PauliSum(np.zeros((1, 6), np.uint8), np.array([3.25]))) - 3.25) < 1e-14
    # D = 1 keeps a product state through entangling gates (largest singular value only)
    m3 = binding.Mps(4, 1, 0.0, bits=[1, 0, 1, 0])
    m3.apply_gate(1, 2, np.kron(np.array([[0.6, 0.8], [-0.8, 0.6]]), np.eye(2)))
    assert list(m3.bond_dims()) == [1, 1, 1, 1, 1]


def test_error_paths_leave_state_unchanged(gpu_lib):
    from paper_2303_03681_amd import binding
    n = 6
    m = binding.Mps(n, 8, 1e-14, bits=hf_bits(n, 3))
    ang = workload_rng(9, 1).uniform(-np.pi, np.pi, size=(2, n, 2))
    _apply(m, fuse_gates(brickwork_gates(n, ang), n))
    plan = binding.PauliSum(np.eye(n, dtype=np.uint8) * 3, np.ones(n))
    e0 = m.expect(plan)
    dims0 = m.bond_dims().copy()
    with pytest.raises(binding.MpsError) as ex:
        m.apply_gate(2, 4, gate_cnot())
    assert ex.value.name == "MPS_ERR_ARG"
    bad = gate_cnot().copy()
    bad[0, 0] = np.nan
    with pytest.raises(binding.MpsError) as ex:
        m.apply_gate(1, 2, bad)
    assert ex.value.name == "MPS_ERR_NONFINITE"
    with pytest.raises(binding.MpsError) as ex:
        m.expect(binding.PauliSum(np.zeros((1, n + 1), np.uint8), np.ones(1)))
    assert ex.value.name == "MPS_ERR_ARG"
    assert list(m.bond_dims()) == list(dims0)
    assert abs(m.expect(plan) - e0) < 1e-13
    with pytest.raises(binding.MpsError) as ex:
        binding.Mps(40, 256, 1e-14, hbm_budget_bytes=1 << 20)
    assert ex.value.name == "MPS_ERR_BUDGET"
    # the sweep limit turns into MPS_ERR_NOCONV and the gate is not applied
    m4 = binding.Mps(8, 16, 1e-14, bits=hf_bits(8, 4), max_jacobi_sweeps=1)
    ang = workload_rng(10, 1).uniform(-np.pi, np.pi, size=(3, 8, 2))
    gates = fuse_gates(brickwork_gates(8, ang), 8)
    q0, q1, u = pack_gates(gates)
    with pytest.raises(binding.MpsError) as ex:
        m4.apply_gates(q0, q1, u)
    assert ex.value.name == "MPS_ERR_NOCONV"


def test_canonicalize_idempotent(gpu_lib):
    from paper_2303_03681_amd import binding
    n = 10
    ang = workload_rng(12, 1).uniform(-np.pi, np.pi, size=(5, n, 2))
    m = binding.Mps(n, 6, 1e-14, bits=hf_bits(n, 5))
    _apply(m, fuse_gates(brickwork_gates(n, ang), n))
    m.canonicalize()
    lam1 = [m.export_site(q)[1] for q in range(n)]
    m.canonicalize()
    assert abs(m.norm() - 1) < 1e-13
    for q in range(n):
        assert np.max(np.abs(m.export_site(q)[1] - lam1[q])) < 1e-12
    for q in range(n):
        B, _ = m.export_site(q)
        g = np.einsum("sab,scb->ac", B, B.conj())
        assert np.max(np.abs(g - np.eye(g.shape[0]))) < 1e-12


def test_expect_without_canonical_form_matches_canonical(gpu_lib):
    """After gates the expectation starts its tries from the identity
    environments of both boundaries and divides by <psi|psi>, leaving the
    state as it is; the values must equal those in exact canonical form
    (diag(lambda^2) and identity roots, Eqs. expec1, rc)."""
    from paper_2303_03681_amd import binding
    n_s = 6
    n = 2 * n_s
    h, g = random_integrals(n_s, workload_rng(71, 0))
    ps = jw_hamiltonian(h, g)
    plan = binding.PauliSum(ps.codes, ps.coeffs)
    ang = workload_rng(71, 1).uniform(-np.pi, np.pi, size=(5, n, 2))
    gates = fuse_gates(brickwork_gates(n, ang), n)
    a = binding.Mps(n, 16, 1e-14, bits=hf_bits(n, n_s))
    b = binding.Mps(n, 16, 1e-14, bits=hf_bits(n, n_s))
    _apply(a, gates)
    _apply(b, gates)
    before = [a.export_site(q) for q in range(n)]
    b.canonicalize()
    for prec, tol in (("c128", 1e-12), ("c64", 2e-5), ("split_f16", 1e-6)):
        ea, pa = a.expect(plan, prec, per_term=True)
        eb, pb = b.expect(plan, prec, per_term=True)
        _say(f"  {prec}: identity environments vs canonical form |dE| {abs(ea - eb):.2e}")
        assert np.max(np.abs(pa - pb)) < tol
    for q in range(n):  # untouched
        B, lam = a.export_site(q)
        assert np.array_equal(B, before[q][0]) and np.array_equal(lam, before[q][1]), q
    assert abs(a.norm() - b.norm()) < 1e-12
    a.canonicalize()
    for q in range(n):
        assert np.max(np.abs(a.export_site(q)[1] - b.export_site(q)[1])) < 1e-12, q
    assert abs(a.expect(plan, "c128") - b.expect(plan, "c128")) < 1e-11


def test_expect_of_unnormalised_imported_state(gpu_lib):
    """A state imported as canonical but scaled by 3 reads <P> unscaled from
    the identity environments once a gate marks it non-canonical: a one-qubit
    identity gate changes nothing but the path."""
    from paper_2303_03681_amd import binding
    n = 6
    o = _canonical_random_oracle(n, 8, 9, layers=3)
    m = binding.Mps(n, 8, 1e-14)
    for q in range(n):
        m.import_site(q, 3.0 * o.B[q] if q == 2 else o.B[q], o.lam[q])
    m.apply_gate(0, -1, np.eye(2))
    codes = np.random.default_rng(5).integers(0, 4, size=(40, n)).astype(np.uint8)
    e, per = m.expect(binding.PauliSum(codes, np.ones(40)), "c128", per_term=True)
    ref = o.expect_terms(codes).real
    assert np.max(np.abs(per - ref)) < 1e-12
    assert abs(m.norm() - 3.0) < 1e-12


def _random_u4(rng):
    z = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _ladder_gates(n, sweeps, seed):
    """Random two-qubit unitaries swept up and down the chain: every gate
    depends on the previous one (batches of one gate)."""
    from workloads.circuits import Gate
    rng = np.random.default_rng(seed)
    gates = []
    for s in range(sweeps):
        bonds = range(n - 1) if s % 2 == 0 else range(n - 2, -1, -1)
        gates += [Gate(q, q + 1, _random_u4(rng)) for q in bonds]
    return gates


@pytest.mark.parametrize("n,D,sweeps", [(9, 8, 4), (12, 32, 3), (14, 64, 3)])
def test_fused_ladder_vs_oracle(gpu_lib, n, D, sweeps):
    """Dependent gates take the fused one-workgroup path (rows of 2 D_l up to
    128, both register widths); bond dimensions, discarded weight and every
    string match the oracle, and the batched path gives the same state."""
    from paper_2303_03681_amd import binding
    _say(f"fused ladder n={n} D={D} sweeps={sweeps}")
    gates = _ladder_gates(n, sweeps, 100 + n)
    bits = hf_bits(n, n // 2)
    o = MpsOracle(n, D, 1e-14, bits)
    o.apply_gates(gates)
    r = np.random.default_rng(n)
    codes = r.integers(0, 4, size=(200, n)).astype(np.uint8)
    coeffs = r.normal(size=200)
    plan = binding.PauliSum(codes, coeffs)
    results = []
    for fused in (True, False):
        m = binding.Mps(n, D, 1e-14, bits=bits)
        m.set_fused_gates(fused)
        _apply(m, gates)
        assert list(m.bond_dims()) == o.bond_dims(), fused
        assert abs(m.discarded_weight() - o.discarded) < 1e-10 * max(1.0, o.discarded)
        e, per = m.expect(plan, "c128", per_term=True)
        results.append((e, per))
    o.canonicalize()
    ref = o.expect_terms(codes).real
    for e, per in results:
        assert np.max(np.abs(per - ref)) < 1e-10
        assert abs(e - math.fsum(coeffs * ref)) < 1e-9
    assert abs(results[0][0] - results[1][0]) < 1e-10


def test_fused_matches_batched_windowed_uccsd(gpu_lib):
    """A 12-qubit windowed UCCSD circuit at D = 64 with cutoff 1e-10 (the
    truncation rule of the 24-qubit workload; only the threshold cuts, the
    discarded weight stays ~1e-20): fused and batched paths match the oracle.
    (At D = 32 the same circuit cuts 1215 times with relative gaps down to
    2e-10 at the cut, where different valid truncations drift apart; such
    cases are not exact-parity cases.)"""
    from paper_2303_03681_amd import binding
    from workloads.circuits import uccsd_gates, uccsd_n_params
    n, ne, D = 12, 6, 64
    h, g = random_integrals(n // 2, workload_rng(4, 0, n))
    ps = jw_hamiltonian(h, g)
    th = workload_rng(4, 1, n).uniform(-0.1, 0.1, uccsd_n_params(n, ne, window=5))
    gates = fuse_gates(uccsd_gates(n, ne, th, window=5), n)
    _say(f"windowed uccsd n={n} gates={len(gates)}")
    o = MpsOracle(n, D, 1e-10, hf_bits(n, ne))
    o.apply_gates(gates)
    o.canonicalize()
    ref = o.expect_terms(ps.codes).real
    e_ref = math.fsum(ps.coeffs * ref)
    plan = binding.PauliSum(ps.codes, ps.coeffs)
    for fused in (True, False):
        m = binding.Mps(n, D, 1e-10, bits=hf_bits(n, ne))
        m.set_fused_gates(fused)
        _apply(m, gates)
        assert list(m.bond_dims()) == o.bond_dims(), fused
        e, per = m.expect(plan, "c128", per_term=True)
        assert np.max(np.abs(per - ref)) < 1e-10, fused
        assert abs(e - e_ref) < 1e-9, fused


@pytest.mark.parametrize("fused", [True, False])
def test_noconv_reports_gates_applied(gpu_lib, fused):
    """A sweep limit of 1 fails the first entangling gate that needs a second
    sweep; the gates before it stay applied and nothing after it is."""
    from paper_2303_03681_amd import binding
    n = 8
    ang = workload_rng(10, 1).uniform(-np.pi, np.pi, size=(3, n, 2))
    gates = fuse_gates(brickwork_gates(n, ang), n)
    q0, q1, u = pack_gates(gates)
    m = binding.Mps(n, 16, 1e-14, bits=hf_bits(n, 4), max_jacobi_sweeps=1)
    m.set_fused_gates(fused)
    with pytest.raises(binding.MpsError) as ex:
        m.apply_gates(q0, q1, u)
    assert ex.value.name == "MPS_ERR_NOCONV"
    k = ex.value.n_done
    assert 0 <= k < len(gates)
    ref = binding.Mps(n, 16, 1e-14, bits=hf_bits(n, 4))
    ref.set_fused_gates(fused)
    if k:
        assert ref.apply_gates(q0[:k], q1[:k], u[:k]) == k
    assert list(m.bond_dims()) == list(ref.bond_dims())
    plan = binding.PauliSum(np.eye(n, dtype=np.uint8) * 3, np.ones(n))
    assert abs(m.expect(plan) - ref.expect(plan)) < 1e-12


def test_boundary_environments_follow_state_changes(gpu_lib):
    """The boundary environments are reused while the state is unchanged and
    recomputed after every change: gates, copies and canonicalisation."""
    from paper_2303_03681_amd import binding
    w = build_config(1)
    n = w.n_qubits
    plan = binding.PauliSum(w.psum.codes, w.psum.coeffs)
    q0, q1, u = pack_gates(w.gates)
    half = len(q0) // 2

    def dense_e(gates):
        return dense_energy(dense_apply_gates(dense_product_state(w.bits), gates), w.psum.codes, w.psum.coeffs)
    m = binding.Mps(n, 16, 1e-14, bits=w.bits)
    m.apply_gates(q0[:half], q1[:half], u[:half])
    e1 = dense_e(w.gates[:half])
    assert abs(m.expect(plan) - e1) < 1e-10
    assert abs(m.expect(plan, "c64") - e1) < 1e-5  # same state, environments reused
    m.apply_gates(q0[half:], q1[half:], u[half:])
    e2 = dense_e(w.gates)
    assert abs(m.expect(plan) - e2) < 1e-10
    other = binding.Mps(n, 16, 1e-14, bits=w.bits)
    other.apply_gates(q0[:10], q1[:10], u[:10])
    other.expect(plan)  # environments of another state
    other.copy_from(m)
    assert abs(other.expect(plan) - e2) < 1e-10
    m.canonicalize()
    assert abs(m.expect(plan) - e2) < 1e-10
    x = np.array([[0, 1], [1, 0]], dtype=complex)
    m.apply_gate(3, -1, x)
    assert abs(m.expect(plan) - dense_e(list(w.gates) + [Gate(3, -1, x)])) < 1e-10
