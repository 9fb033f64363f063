"""GPU: HIP-graph replay of the expectation.  Every replay must equal the
eager path bitwise, with eager work and synchronisations between replays,
after gates change the state (fresh site buffers, same or new bond dims), in
both root kinds (boundary environments, exact canonical form) and together
with tile autotuning."""

import numpy as np
import pytest

from workloads import brickwork_gates, fuse_gates, hf_bits, jw_hamiltonian, pack_gates, \
    random_integrals, workload_rng

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _setup(binding, n_s=6, D=32, layers=5, seed=91):
    n = 2 * n_s
    h, g = random_integrals(n_s, workload_rng(seed, 0))
    ps = jw_hamiltonian(h, g)
    ang = workload_rng(seed, 1).uniform(-np.pi, np.pi, size=(layers, n, 2))
    gates = pack_gates(fuse_gates(brickwork_gates(n, ang), n))
    return n, binding.PauliSum(ps.codes, ps.coeffs), gates


def _twins(binding, n, D, gates):
    a = binding.Mps(n, D, 1e-12, bits=hf_bits(n, n // 2))
    b = binding.Mps(n, D, 1e-12, bits=hf_bits(n, n // 2))
    a.apply_gates(*gates)
    b.apply_gates(*gates)
    b.set_graphs(True)
    return a, b


def test_graph_replays_equal_eager(gpu_lib):
    import torch
    from paper_2303_03681_amd import binding
    n, plan, gates = _setup(binding)
    for prec in ("c128", "c64", "split_f16"):
        a, b = _twins(binding, n, 32, gates)
        _say(f"graphs {prec}")
        b.set_timing(True)
        ref = a.expect(plan, prec, per_term=True)[1]
        x = torch.ones(1 << 20, device="cuda")
        for rep in range(4):
            e, p = b.expect(plan, prec, per_term=True)
            assert np.array_equal(p, ref), (prec, rep)
            x.mul_(1.0001)                        # eager work between replays
            a.expect(plan, prec)                  # and another handle's launches
            torch.cuda.synchronize()
        assert b.timing()["graph_launches"] == 4  # first call captures, every call replays
        # gates change the state: the replay must read the new sites
        q0, q1, u = gates
        k = len(q0) // 3
        for m in (a, b):
            m.apply_gates(q0[:k], q1[:k], u[:k])
        assert list(a.bond_dims()) == list(b.bond_dims())
        assert np.array_equal(b.expect(plan, prec, per_term=True)[1], a.expect(plan, prec, per_term=True)[1])
        # exact canonical form: the other root kind
        a.canonicalize()
        b.canonicalize()
        for _ in range(2):
            assert np.array_equal(b.expect(plan, prec, per_term=True)[1],
                                  a.expect(plan, prec, per_term=True)[1])


def test_graphs_with_autotune_and_forced_tiles(gpu_lib):
    from paper_2303_03681_amd import binding
    binding.autotune_reset()
    n, plan, gates = _setup(binding, n_s=5, D=24, seed=92)
    a, b = _twins(binding, n, 24, gates)
    ref = a.expect(plan, "c64", per_term=True)[1]
    b.set_autotune(True)
    b.set_timing(True)
    for _ in range(3):  # tunes eagerly, then captures and replays
        assert np.array_equal(b.expect(plan, "c64", per_term=True)[1], ref)
    assert b.timing()["graph_launches"] == 2
    for t in (1, 3):
        b.set_env_tile(t)  # re-captured with the forced tile
        assert np.array_equal(b.expect(plan, "c64", per_term=True)[1], ref)
    b.set_env_tile(-1)
    b.set_graphs(False)
    assert np.array_equal(b.expect(plan, "c64", per_term=True)[1], ref)
    binding.autotune_reset()
