"""GPU: windowed qubit-ADAPT on the 8-qubit Hamiltonian (pool derivatives
against the commutator formula on the oracle's dense state, energies
lowered and above exact diagonalisation) and the bond-dimension rule on a
16-qubit windowed UCCSD state (largest D without truncation equals the dense
energy)."""

import numpy as np
import pytest

from oracle import dense_apply_gates, dense_apply_pauli, dense_energy, dense_pauli_matrix, \
    dense_product_state
from workloads import build_config, fuse_gates, hf_bits, jw_hamiltonian, pack_gates, \
    qubit_adapt_pool, random_integrals, uccsd_gates, workload_rng
from workloads.circuits import pauli_exponential_gates, uccsd_n_params

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_qubit_adapt_iterations(gpu_lib):
    from paper_2303_03681_amd import binding
    from paper_2303_03681_amd.adapt import QubitAdapt
    w = build_config(1, with_gates=False)
    n = w.n_qubits
    plan = binding.PauliSum(w.psum.codes, w.psum.coeffs)
    pool = qubit_adapt_pool(n, 5)
    ad = QubitAdapt(n, plan, pool, 16, bits=w.bits, batch=32)
    H = sum(c * dense_pauli_matrix(code) for code, c in zip(w.psum.codes, w.psum.coeffs))
    e_exact = float(np.linalg.eigvalsh(H)[0])
    prev = None
    for it in range(3):
        ad.prepare()
        g = ad.pool_gradients()
        psi = dense_product_state(w.bits)
        for a, t in zip(ad.ops, ad.theta):
            psi = dense_apply_gates(psi, pauli_exponential_gates(pool[a], float(t)))
        hpsi = sum(c * dense_apply_pauli(psi, code) for code, c in zip(w.psum.codes, w.psum.coeffs))
        comm = np.array([-2.0 * np.vdot(hpsi.ravel(), dense_apply_pauli(psi, P).ravel()).imag for P in pool])
        _say(f"iteration {it}: max |g| {np.max(np.abs(g)):.4f}, |g - commutator| {np.max(np.abs(g - comm)):.1e}")
        assert np.max(np.abs(g - comm)) < 1e-10
        rec = ad.iterate(opt_steps=4, lr=0.2)
        assert abs(abs(comm[rec["selected"]]) - np.max(np.abs(comm))) < 1e-10
        _say(f"  selected {rec['selected']}, E {rec['energy_before']:.6f} -> {rec['energy_after']:.6f}")
        assert rec["energy_after"] < rec["energy_before"] and rec["energy_after"] >= e_exact - 1e-9
        if prev is not None:
            assert rec["energy_before"] == pytest.approx(prev, abs=1e-10)
        prev = rec["energy_after"]
    ad.close()


def test_bond_dimension_rule(gpu_lib):
    from paper_2303_03681_amd import binding
    from paper_2303_03681_amd.adapt import bond_dimension_scan, select_bond_dimension
    n_s, n, ne = 8, 16, 8
    h, g = random_integrals(n_s, workload_rng(97, 0))
    ps = jw_hamiltonian(h, g)
    theta = workload_rng(97, 1).uniform(-0.3, 0.3, size=uccsd_n_params(n, ne, window=3))
    gl = uccsd_gates(n, ne, theta, window=3)
    gates = pack_gates(fuse_gates(gl, n))
    plan = binding.PauliSum(ps.codes, ps.coeffs)
    bonds = [4, 8, 16, 32, 64, 96, 128, 256]
    es = bond_dimension_scan(n, gates, plan, hf_bits(n, ne), bonds)
    _say("D scan: " + ", ".join(f"{d}: {e:.8f}" for d, e in zip(bonds, es)))
    psi = dense_apply_gates(dense_product_state(hf_bits(n, ne)), gl)
    e_dense = dense_energy(psi, ps.codes, ps.coeffs)
    assert abs(es[-1] - e_dense) < 1e-9  # D = 256 = 2^(n/2): no truncation
    d = select_bond_dimension(bonds, es, 1e-3)
    _say(f"selected D = {d}")
    assert d is not None
    i = bonds.index(d)
    assert abs(es[i] - es[i + 1]) < 1e-3
    assert all(abs(es[j] - es[j + 1]) >= 1e-3 for j in range(i))
