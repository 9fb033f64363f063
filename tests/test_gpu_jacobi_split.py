"""GPU: the batched gate SVDs (Algorithm 1 rounds of the register and
wide-row kernels) split over streams.  Each matrix goes through the same
rotation rounds on one, two or three streams, so the state after a brickwork
circuit whose middle bonds reach D = 256 (512 x 512 SVDs, register kernels)
or D = 512 (rows 1024 long, wide-row kernel), with enough items per layer to
split, must agree site by site (and in energy for D = 256)."""

import time

import numpy as np
import pytest

from workloads import brickwork_gates, fuse_gates, hf_bits, jw_hamiltonian, pack_gates, \
    random_integrals, workload_rng

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("n_s,D,layers", [(18, 256, 9), (15, 512, 11)])
def test_split_rounds_match_one_stream(gpu_lib, n_s, D, layers):
    from paper_2303_03681_amd import binding
    n = 2 * n_s
    ang = workload_rng(97, 1).uniform(-np.pi, np.pi, size=(layers, n, 2))
    gates = pack_gates(fuse_gates(brickwork_gates(n, ang), n))
    plan = None
    if D <= 256:
        h, g = random_integrals(n_s, workload_rng(97, 0))
        ps = jw_hamiltonian(h, g)
        plan = binding.PauliSum(ps.codes, ps.coeffs)
    out = {}
    for groups in (1, 2, 3):
        _say(f"brickwork n={n} layers={layers} D={D} jacobi_groups={groups}")
        m = binding.Mps(n, D, 1e-12, bits=hf_bits(n, n_s))
        m.set_jacobi_groups(groups)
        t0 = time.perf_counter()
        m.apply_gates(*gates)
        dt = time.perf_counter() - t0
        dims = m.bond_dims()
        sites = [m.export_site(q) for q in range(n)]
        e = m.expect(plan, "c128") if plan is not None else 0.0
        out[groups] = (dims, sites, e)
        _say(f"  gates {dt:.3f} s, max bond {dims.max()}, E = {e:.15f}")
        m.close()
    d0, s0, e0 = out[1]
    assert d0.max() == D
    for groups in (2, 3):
        d1, s1, e1 = out[groups]
        assert np.array_equal(d0, d1)
        worst = 0.0
        for (b0, l0), (b1, l1) in zip(s0, s1):
            worst = max(worst, float(np.max(np.abs(b0 - b1))), float(np.max(np.abs(l0 - l1))))
        _say(f"  groups {groups}: max site difference {worst:.2e}, |dE| {abs(e0 - e1):.2e}")
        assert worst <= 1e-12
        assert abs(e0 - e1) <= 1e-12
    m = binding.Mps(4, 4, 1e-12)
    for bad in (0, 4):
        with pytest.raises(binding.MpsError):
            m.set_jacobi_groups(bad)
    m.close()
