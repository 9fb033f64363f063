"""GPU: fragment 1- and 2-RDMs through mps_expect_pauli_rows against the
oracle's ladder-operator RDMs (exact 8-qubit UCCSD state) and against the
oracle MPS's string values on a truncated state; row-array validation."""

import math

import numpy as np
import pytest

from oracle import MpsOracle, dense_apply_gates, dense_product_state, dense_rdm1, dense_rdm2
from workloads import brickwork_gates, build_config, fuse_gates, hf_bits, pack_gates, workload_rng

pytestmark = pytest.mark.gpu


def test_rdms_of_uccsd_state_vs_ladder_operators(gpu_lib):
    from paper_2303_03681_amd import binding
    from paper_2303_03681_amd.rdm import RdmEvaluator
    w = build_config(1)
    n = w.n_qubits
    m = binding.Mps(n, 16, 1e-14, bits=w.bits)
    m.apply_gates(*pack_gates(w.gates))
    psi = dense_apply_gates(dense_product_state(w.bits), w.gates)
    ev = RdmEvaluator(n)
    g1_ref, g2_ref = dense_rdm1(psi), dense_rdm2(psi)
    for prec, tol in (("c128", 1e-11), ("c64", 2e-6)):
        g1 = ev.one_rdm(m, prec)
        g2 = ev.two_rdm(m, prec)
        print(f"{prec}: |d gamma| {np.max(np.abs(g1 - g1_ref)):.2e}, |d Gamma| {np.max(np.abs(g2 - g2_ref)):.2e}",
              flush=True)
        assert np.max(np.abs(g1 - g1_ref)) < tol
        assert np.max(np.abs(g2 - g2_ref)) < tol
    ne = int(np.sum(w.bits))
    assert abs(np.trace(ev.one_rdm(m)) - ne) < 1e-11


def test_rows_on_truncated_state_vs_oracle_mps(gpu_lib):
    from paper_2303_03681_amd import binding
    from paper_2303_03681_amd.rdm import RdmEvaluator
    n = 10
    ang = workload_rng(95, 1).uniform(-np.pi, np.pi, size=(5, n, 2))
    gates = fuse_gates(brickwork_gates(n, ang), n)
    bits = hf_bits(n, 5)
    m = binding.Mps(n, 8, 1e-14, bits=bits)
    m.apply_gates(*pack_gates(gates))
    o = MpsOracle(n, 8, 1e-14, bits)
    o.apply_gates(gates)
    o.canonicalize()
    ev = RdmEvaluator(n)
    for rows, plan, got in ((ev.r1, ev.p1, ev.one_rdm(m).ravel()),):
        per = o.expect_terms(rows.strings.codes).real
        ref = np.array([math.fsum(rows.vals[a:b] * per[rows.cols[a:b]])
                        for a, b in zip(rows.row_ptr[:-1], rows.row_ptr[1:])])
        assert np.max(np.abs(got - (ref[0::2] + 1j * ref[1::2]))) < 1e-10
    g2 = ev.two_rdm(m)
    per = o.expect_terms(ev.r2.strings.codes).real
    r = ev.r2
    ref = np.array([math.fsum(r.vals[a:b] * per[r.cols[a:b]]) for a, b in zip(r.row_ptr[:-1], r.row_ptr[1:])])
    p, q, s, t = r.elements.T
    assert np.max(np.abs(g2[p, q, s, t] - (ref[0::2] + 1j * ref[1::2]))) < 1e-10


def test_rows_argument_checks(gpu_lib):
    from paper_2303_03681_amd import binding
    m = binding.Mps(4, 4, 1e-14)
    plan = binding.PauliSum(np.array([[3, 0, 0, 0], [0, 3, 0, 0]], np.uint8), np.ones(2))
    out = m.expect_rows(plan, [0, 2, 3], [0, 1, 1], [1.0, 2.0, -1.0])
    assert np.allclose(out, [3.0, -1.0])
    assert m.expect_rows(plan, [0], [], []).size == 0
    for rp, cols in (([1, 2], [0, 1]), ([0, 2, 1], [0, 1]), ([0, 1], [2])):
        with pytest.raises(binding.MpsError) as ex:
            m.expect_rows(plan, rp, cols, np.ones(len(cols)))
        assert ex.value.name == "MPS_ERR_ARG"
