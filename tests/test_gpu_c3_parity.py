"""GPU: the 50-qubit brickwork evaluation's own code path against the FP64
oracle.

Two reduced cases of the same recipe (random-integral JW Hamiltonian sampled
uniformly, brickwork ansatz with angles U(-pi, pi), cutoff 1e-14), with the
oracle's results stored by tests/golden/make_c3_reduced.py (oracle/ and
workloads/ only), run with the settings of the benchmark (tile autotuning on,
batched Jacobi rounds in two item groups):

  * 36 qubits, 12 layers, D = 256, 4096 strings: 512 x 512 gate SVDs in
    multi-item register rounds split over item groups, saturated D = 256
    environment products with tuned tiles, split-K closing traces;
  * 28 qubits, 13 layers, D = 512, 512 strings: 1024 x 1024 gate SVDs in the
    wide-row rounds and the D = 512 products of Eqs. (C) and (Bl).

Every cut at the bond cap has a relative gap far above round-off (smallest
4e-4 at 36 qubits; recorded in the golden file), so the truncated state is
an exact-parity quantity: bond dimensions must be equal, the discarded
weight equal to 1e-10 relative, every string equal to 1e-10 and the energy
to 1e-9 in complex128.  The FP32 and split-16-bit environment paths are
compared with complex128 on the same state.

The full 50-qubit state after all 980 gates is then exported and 64 of its
strings (the largest |<P>| and random ones) are recomputed by the oracle's
full contraction (identity transfers from the left boundary, explicit right
boundary, no gauge assumed)."""

import json
import os
import time

import numpy as np
import pytest

from workloads import build_config, pack_gates

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_reduced.json")


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


def _bench_like(binding, n, D, cutoff, bits):
    m = binding.Mps(n, D, cutoff, bits=bits)
    m.set_autotune(True)
    m.set_jacobi_groups(2)
    m.set_timing(True)
    return m


@pytest.mark.parametrize("case", ["36q_D256", "28q_D512"])
def test_c3_recipe_vs_oracle(gpu_lib, gold, case):
    from paper_2303_03681_amd import binding
    ref = gold[case]
    w = build_config(3, n_spatial=ref["n_spatial"], layers=ref["layers"], n_strings=ref["n_strings"])
    assert len(w.gates) == ref["n_gates"] and w.psum.n_terms == ref["n_terms"]
    D = ref["max_bond"]
    _say(f"C3 recipe {case}: {w.n_qubits} q, {len(w.gates)} gates, D={D}, {w.psum.n_terms} strings; "
         f"oracle cap cuts {ref['cap_cuts']}, smallest relative gap {ref['min_cap_gap']:.2e}")
    m = _bench_like(binding, w.n_qubits, D, w.spec.cutoff, w.bits)
    q0, q1, u = pack_gates(w.gates)
    t0 = time.perf_counter()
    assert m.apply_gates(q0, q1, u) == len(q0)
    tg = time.perf_counter() - t0
    tm = m.timing()
    dims = m.bond_dims()
    disc = m.discarded_weight()
    _say(f"  gates {tg:.2f} s; multi-launch SVDs {tm['jacobi_multi_items']} "
         f"(wide rows {tm['jacobi_wide_items']}), batches split over groups {tm['jacobi_split_batches']}")
    # the benchmark's paths were taken
    assert tm["jacobi_split_batches"] > 0
    if D == 512:
        assert tm["jacobi_wide_items"] > 0
    assert list(dims) == ref["bond_dims"]
    assert abs(disc - ref["discarded_weight"]) <= 1e-10 * ref["discarded_weight"]
    plan = binding.PauliSum(w.psum.codes, w.psum.coeffs)
    e128, per = m.expect(plan, "c128", per_term=True)
    vals = np.array(ref["values"])
    d_str = float(np.max(np.abs(per - vals)))
    _say(f"  c128: |dE| {abs(e128 - ref['energy']):.2e}, max |d<P>| {d_str:.2e}, "
         f"|d disc| {abs(disc - ref['discarded_weight']):.2e}")
    assert d_str <= 1e-10
    assert abs(e128 - ref["energy"]) <= 1e-9
    # lower-precision environments on the same state, against complex128
    bounds = {"c64": 1e-6, "split_f16": 1e-6, "split_bf16": 1e-5}
    for prec, bound in bounds.items():
        e_p, per_p = m.expect(plan, prec, per_term=True)
        _say(f"  {prec}: |E - E_c128| {abs(e_p - e128):.2e}, max |d<P>| {np.max(np.abs(per_p - per)):.2e}")
        assert abs(e_p - e128) <= bound
        assert np.max(np.abs(per_p - per)) <= 10 * bound
    m.close()
    plan.close()


def test_c3_full_state_strings_vs_oracle(gpu_lib):
    """The full 50-qubit, 980-gate, D = 256 state of the benchmark: 64 strings
    of the 2^18 sample against the oracle's full contraction of the exported
    state."""
    from oracle import MpsOracle
    from paper_2303_03681_amd import binding
    t0 = time.perf_counter()
    w = build_config(3)
    _say(f"C3 full: workload built in {time.perf_counter() - t0:.1f} s")
    m = _bench_like(binding, w.n_qubits, w.spec.max_bond, w.spec.cutoff, w.bits)
    q0, q1, u = pack_gates(w.gates)
    assert m.apply_gates(q0, q1, u) == len(q0)
    plan = binding.PauliSum(w.psum.codes, w.psum.coeffs)
    e128, per = m.expect(plan, "c128", per_term=True)
    dims = m.bond_dims()
    _say(f"C3 full: E_c128 = {e128:.15f}, max bond {dims.max()}, discarded {m.discarded_weight():.4f}")
    assert dims.max() == w.spec.max_bond
    o = MpsOracle(w.n_qubits, w.spec.max_bond, w.spec.cutoff)
    o.B = []
    for q in range(w.n_qubits):
        b, lam = m.export_site(q)
        o.B.append(b)
    rng = np.random.default_rng(2024)
    top = np.argsort(-np.abs(per))[:32]
    rest = rng.choice(np.setdiff1d(np.arange(w.psum.n_terms), top), size=32, replace=False)
    worst = 0.0
    t0 = time.perf_counter()
    for k in np.concatenate([top, rest]):
        ref = o.expect_pauli_full(w.psum.codes[k])
        worst = max(worst, abs(per[k] - ref.real))
    _say(f"C3 full: 64 strings (largest |<P>| {np.abs(per[top[0]]):.3e}) vs oracle full contraction: "
         f"max |d<P>| {worst:.2e} ({time.perf_counter() - t0:.0f} s)")
    assert worst <= 1e-10
    m.close()
    plan.close()
