"""GPU: the environment GEMM tile autotuner.  Every tile shape must give
bitwise the same per-string values (each output element accumulates its K
range in the same order of 16x16x4 steps); tuning must only pick among them
and record its measurements."""

import numpy as np
import pytest

from workloads import brickwork_gates, fuse_gates, hf_bits, jw_hamiltonian, pack_gates, \
    random_integrals, workload_rng

pytestmark = pytest.mark.gpu


def _state(binding, n_s=7, D=48, layers=6):
    n = 2 * n_s
    h, g = random_integrals(n_s, workload_rng(81, 0))
    ps = jw_hamiltonian(h, g)
    ang = workload_rng(81, 1).uniform(-np.pi, np.pi, size=(layers, n, 2))
    m = binding.Mps(n, D, 1e-12, bits=hf_bits(n, n_s))
    m.apply_gates(*pack_gates(fuse_gates(brickwork_gates(n, ang), n)))
    return m, binding.PauliSum(ps.codes, ps.coeffs)


def test_every_tile_shape_bitwise_equal(gpu_lib):
    from paper_2303_03681_amd import binding
    m, plan = _state(binding)
    for prec in ("c128", "c64"):
        e0, p0 = m.expect(plan, prec, per_term=True)
        for t in range(8):
            m.set_env_tile(t)
            e, p = m.expect(plan, prec, per_term=True)
            assert np.array_equal(p, p0) and e == e0, (prec, t)
        m.set_env_tile(-1)
    with pytest.raises(binding.MpsError):
        m.set_env_tile(8)


def test_autotune_table_and_results(gpu_lib):
    from paper_2303_03681_amd import binding
    binding.autotune_reset()
    assert binding.autotune_table() == []
    m, plan = _state(binding)
    ref = {p: m.expect(plan, p, per_term=True)[1] for p in ("c128", "c64")}
    m.set_autotune(True)
    for prec in ("c128", "c64"):
        tuned_pass = m.expect(plan, prec, per_term=True)[1]   # tunes unknown classes
        after = m.expect(plan, prec, per_term=True)[1]        # uses the table
        assert np.array_equal(tuned_pass, ref[prec]) and np.array_equal(after, ref[prec])
    rows = binding.autotune_table()
    assert {r["prec"] for r in rows} == {"c128", "c64"}
    assert {r["half"] for r in rows} == {1, 2}
    shapes = ["64x64x16", "32x32x16", "128x64x16", "64x128x16", "64x64x32", "32x64x16", "128x128x16",
              "128x128x8"]
    for r in rows:
        assert 0 <= r["tile"] < 8 and r["shape"] == shapes[r["tile"]]
        assert len(r["ms"]) == 8 and all(x > 0 for x in r["ms"])
        assert r["ms"][r["tile"]] == min(r["ms"])
    # a second handle of the same shapes finds every class in the table
    m2, plan2 = _state(binding)
    m2.set_autotune(True)
    m2.expect(plan2, "c64")
    assert len(binding.autotune_table()) == len(rows)
    binding.autotune_reset()
