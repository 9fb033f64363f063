"""GPU: mps_to_statevector (the contraction of Eq. mps on the device) against
the oracle's dense statevector, with no truncation: the 8-qubit UCCSD
workload and a 12-qubit brickwork circuit, before and after
canonicalisation; the qubit-count limit is an argument error."""

import numpy as np
import pytest

from oracle import dense_apply_gates, dense_product_state
from workloads import brickwork_gates, build_config, fuse_gates, hf_bits, pack_gates, workload_rng

pytestmark = pytest.mark.gpu


def _check(m, psi_ref, tol=1e-12):
    psi = m.to_statevector()
    err = float(np.max(np.abs(psi - psi_ref.ravel())))
    print(f"  max |d psi| {err:.2e}", flush=True)
    assert err <= tol


def test_statevector_uccsd_8q(gpu_lib):
    from paper_2303_03681_amd import binding
    w = build_config(1)
    print("statevector: 8q UCCSD", flush=True)
    m = binding.Mps(w.n_qubits, 16, 1e-14, bits=w.bits)
    m.apply_gates(*pack_gates(w.gates))
    ref = dense_apply_gates(dense_product_state(w.bits), w.gates)
    _check(m, ref)
    m.canonicalize()
    _check(m, ref)
    m.close()


def test_statevector_brickwork_12q(gpu_lib):
    from paper_2303_03681_amd import binding
    n = 12
    ang = workload_rng(55, 1).uniform(-np.pi, np.pi, size=(5, n, 2))
    gates = fuse_gates(brickwork_gates(n, ang), n)
    bits = hf_bits(n, 6)
    print("statevector: 12q brickwork, 5 layers, D = 64 (exact)", flush=True)
    m = binding.Mps(n, 64, 1e-14, bits=bits)
    m.apply_gates(*pack_gates(gates))
    ref = dense_apply_gates(dense_product_state(bits), gates)
    _check(m, ref)
    # product state and a single site
    m.reset(bits)
    _check(m, dense_product_state(bits))
    m.close()
    one = binding.Mps(1, 1, 1e-14, bits=np.array([1], np.uint8))
    _check(one, np.array([0.0, 1.0], complex))
    one.close()


def test_statevector_limit(gpu_lib):
    """27 qubits exceed the limit: MPS_ERR_ARG before any output is written
    (a 4-element buffer is passed, so a write would be out of bounds on the
    host side only; the call must fail on the qubit count first)."""
    from paper_2303_03681_amd import binding
    m = binding.Mps(27, 2, 1e-14)
    psi = np.zeros(4, np.complex128)
    with pytest.raises(binding.MpsError) as err:
        binding._check(binding.load().mps_to_statevector(m._h, binding._ptr(psi.view(np.float64))))
    assert err.value.name == "MPS_ERR_ARG"
    assert not np.any(psi)
    m.close()
