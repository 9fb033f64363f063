"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point of include/mps.h, and its Pauli planner (host C++) produces
plans whose tries, evaluated with numpy transfer matrices on an oracle MPS,
reproduce every per-string expectation."""

import ctypes

import numpy as np
import pytest

from paper_2303_03681_amd import binding
from oracle import MpsOracle
from oracle.mps import _PAULI
from workloads import brickwork_gates, build_config, fuse_gates, hf_bits, jw_hamiltonian, \
    random_integrals, workload_rng


def test_library_exports_every_header_symbol():
    lib = binding.load()
    syms = binding.header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    raw = ctypes.CDLL(binding.LIB_PATH)
    for s in syms:
        getattr(raw, s)


def _eval_plan(plan, m: MpsOracle):
    lpar, lsite, llet = plan["left"]
    rpar, rsite, rlet = plan["right"]
    cb, cl, cr = plan["close"]
    Lenv, Renv = {}, {}

    def lget(ref):
        if ref < 0:
            return np.diag(m.lam[-ref - 1] ** 2).astype(complex)
        return Lenv[ref]

    def rget(ref):
        if ref < 0:
            d = m.lam[-ref - 1].size
            return np.eye(d, dtype=complex)
        return Renv[ref]

    for i in range(lpar.size):
        assert lpar[i] < i  # parents come first
        Lenv[i] = m._transfer(lget(lpar[i]), int(lsite[i]), int(llet[i]))
    for i in range(rpar.size):
        assert rpar[i] < i
        B = m.B[int(rsite[i])]
        sig = _PAULI[int(rlet[i])]
        R = rget(rpar[i])
        out = np.zeros((B.shape[1], B.shape[1]), dtype=complex)
        for s in range(2):
            for sp in range(2):
                if sig[s, sp] != 0:
                    out += sig[s, sp] * (B[sp] @ R @ B[s].conj().T)
        Renv[i] = out
    return np.array([np.trace(lget(cl[k]) @ rget(cr[k])) for k in range(cb.size)])


@pytest.mark.parametrize("n_s,layers,D", [(4, 3, 8), (5, 4, 6)])
def test_planner_reproduces_per_string_expectations(n_s, layers, D):
    n = 2 * n_s
    h, g = random_integrals(n_s, workload_rng(40 + n_s, 0))
    ps = jw_hamiltonian(h, g)
    ang = workload_rng(40 + n_s, 1).uniform(-np.pi, np.pi, size=(layers, n, 2))
    m = MpsOracle(n, D, 1e-14, hf_bits(n, n_s))
    m.apply_gates(fuse_gates(brickwork_gates(n, ang), n))
    m.canonicalize()
    plan = binding.PauliSum(ps.codes, ps.coeffs)
    ex = plan.export()
    got = _eval_plan(ex, m)
    ref = m.expect_terms(ps.codes)
    assert np.max(np.abs(got - ref)) < 1e-12
    st = plan.stats()
    # sharing: far fewer transfer updates than a per-string walk
    walk = sum(int(np.nonzero(c)[0][-1] - np.nonzero(c)[0][0] + 1) for c in ps.codes if c.any())
    assert st["left_updates"] + st["right_updates"] < walk


def test_planner_random_strings_and_edge_cases():
    n = 7
    r = np.random.default_rng(3)
    codes = r.integers(0, 4, size=(60, n)).astype(np.uint8)
    codes[0] = 0                      # identity
    codes[1] = [3, 0, 0, 0, 0, 0, 0]  # first qubit only
    codes[2] = [0, 0, 0, 0, 0, 0, 2]  # last qubit only
    codes[3] = [1, 0, 0, 0, 0, 0, 1]  # longest identity run
    codes[4] = [2, 2, 2, 2, 2, 2, 2]  # no identity
    coeffs = r.normal(size=60)
    ang = r.uniform(-np.pi, np.pi, size=(3, n, 2))
    m = MpsOracle(n, 5, 1e-14, hf_bits(n, 3))
    m.apply_gates(brickwork_gates(n, ang))
    m.canonicalize()
    plan = binding.PauliSum(codes, coeffs)
    got = _eval_plan(plan.export(), m)
    ref = m.expect_terms(codes)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_planner_rejects_bad_input():
    with pytest.raises(binding.MpsError) as e:
        binding.PauliSum(np.full((2, 3), 7, np.uint8), np.ones(2))
    assert e.value.name == "MPS_ERR_ARG"
    with pytest.raises(binding.MpsError):
        binding.PauliSum(np.zeros((1, 3), np.uint8), np.array([np.nan]))


def test_planner_empty_sum():
    plan = binding.PauliSum(np.zeros((0, 5), np.uint8), np.zeros(0))
    assert plan.stats()["closes"] == 0


def test_planner_c3_scale_stats():
    """The 50-qubit sampled Hamiltonian plans to well under one transfer
    update per string (prefix/suffix sharing meeting at one bond)."""
    w = build_config(3, with_gates=False, n_strings=1 << 17)
    plan = binding.PauliSum(w.psum.codes, w.psum.coeffs)
    st = plan.stats()
    assert st["left_updates"] + st["right_updates"] < 0.4 * w.psum.n_terms
    assert 10 <= st["meet_bond"] <= 40


def test_autotune_table_host_only():
    """The tuning table is host state: empty after a reset, without a GPU."""
    from paper_2303_03681_amd import binding
    binding.autotune_reset()
    assert binding.autotune_table() == []
