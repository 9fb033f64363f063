"""Request-loop policy of the serving engine, on the CPU with a fake device
backend: admission by slots and memory budget, per-fragment update order,
eviction of idle fragments, isolation of a failed request, and arrivals
joining between gate chunks (continuous batching)."""

import numpy as np
import pytest

from paper_2303_03681_amd.serving import Fragment, Request, Server, estimate_bytes, make_requests


class FakeError(RuntimeError):
    pass


class FakeBackend:
    def __init__(self, bytes_per_fragment=100, fail=None):
        self.bytes = bytes_per_fragment
        self.live = {}          # id(handle) -> fid
        self.max_live_bytes = 0
        self.chunk_sizes = []
        self.chunk_members = []
        self.fail = fail        # (fid, update, gate) that fails
        self.current = {}

    def create(self, frag):
        h = {"fid": frag.fid, "applied": 0}
        self.live[id(h)] = frag.fid
        self.max_live_bytes = max(self.max_live_bytes, len(self.live) * self.bytes)
        return h

    def plan_updates(self, frag):
        return 10

    def reset(self, h, frag):
        h["applied"] = 0

    def apply_chunk(self, items):
        self.chunk_sizes.append(len(items))
        self.chunk_members.append(tuple(sorted(it[0]["fid"] for it in items)))
        done = []
        err = None
        for h, q0, q1, u in items:
            k = len(q0)
            if self.fail and h["fid"] == self.fail[0] and h.get("update") == self.fail[1]:
                k = 0
                err = FakeError("gate failed")
            h["applied"] += k
            done.append(k)
        if err is not None:
            err.n_done = np.array(done)
            raise err
        return np.array(done)

    def expect(self, h, frag):
        return float(frag.fid) + 0.001 * h["applied"]

    def apply_all(self, h, frag, update):
        h["applied"] += len(frag.updates[update][0])

    def device_bytes(self, h):
        return self.bytes

    def destroy(self, h):
        self.live.pop(id(h), None)


def _frags(n, gates_per_update=(700, 300), n_updates=3, qubits=12, bond=32):
    out = []
    for fid in range(n):
        ups = []
        for u in range(n_updates):
            g = gates_per_update[(fid + u) % len(gates_per_update)]
            ups.append((np.zeros(g, np.int32), np.full(g, 1, np.int32), np.zeros((g, 16, 2))))
        out.append(Fragment(fid, qubits, bond, 1e-10, np.zeros(qubits, np.uint8),
                            np.zeros((3, qubits), np.uint8), np.ones(3), ups, est_bytes=100))
    return out


def test_all_complete_in_update_order():
    frags = _frags(4)
    reqs = make_requests(4, 3, rate=2000.0, rng=np.random.default_rng(1))
    be = FakeBackend()
    rep = Server(frags, be, max_active=3, chunk=256, chunk_s=1e9, max_chunk=256).run(reqs)
    assert rep.completed == len(reqs)
    by_frag = {}
    for r in rep.requests:
        by_frag.setdefault(r.fid, []).append(r)
    for fid, rs in by_frag.items():
        rs.sort(key=lambda r: r.update)
        assert [r.update for r in rs] == [0, 1, 2]
        for a, b in zip(rs, rs[1:]):
            assert b.admitted >= a.finish - 1e-9  # next update only after the previous
    assert max(be.chunk_sizes) <= 3
    # energies are the fake's function of (fragment, gates of that update)
    for r in rep.requests:
        g = frags[r.fid].updates[r.update][0].size
        assert r.energy == pytest.approx(r.fid + 0.001 * g)
    s = rep.summary()
    assert s["completed"] == len(reqs) and s["latency_ms"]["p99"] >= s["latency_ms"]["p50"]


def test_budget_evicts_idle_fragments():
    frags = _frags(5)
    reqs = make_requests(5, 2, rate=5000.0, rng=np.random.default_rng(2))
    be = FakeBackend(bytes_per_fragment=100)
    rep = Server(frags, be, max_active=8, hbm_budget=250, chunk=128).run(reqs)
    assert rep.completed == len(reqs)
    assert be.max_live_bytes <= 250
    assert rep.evictions > 0


def test_budget_too_small_is_reported():
    frags = _frags(1)
    frags[0].est_bytes = 1000
    reqs = [Request(0, 0, 0, 0.0)]
    with pytest.raises(RuntimeError, match="cannot be admitted"):
        Server(frags, FakeBackend(), hbm_budget=10).run(reqs)


def test_arrivals_join_between_chunks():
    """A request arriving while others are mid-circuit is admitted at the next
    chunk boundary: chunk memberships change while earlier requests run."""
    frags = _frags(3, gates_per_update=(3000,), n_updates=1)

    class SlowBackend(FakeBackend):
        def apply_chunk(self, items):
            import time
            time.sleep(0.01)
            return super().apply_chunk(items)
    be = SlowBackend()
    reqs = [Request(0, 0, 0, 0.0), Request(1, 1, 0, 0.03), Request(2, 2, 0, 0.06)]
    rep = Server(frags, be, max_active=8, chunk=256, max_chunk=256).run(reqs)
    assert rep.completed == 3
    members = be.chunk_members
    assert (0,) in members and (0, 1) in members and (0, 1, 2) in members


def test_failed_gate_isolated_to_its_request():
    frags = _frags(3, gates_per_update=(500,), n_updates=1)

    class FailOne(FakeBackend):
        def apply_chunk(self, items):
            for h, *_ in items:
                h["update"] = 0
            return super().apply_chunk(items)
    be = FailOne(fail=(1, 0, 0))
    reqs = [Request(i, i, 0, 0.0) for i in range(3)]
    rep = Server(frags, be, max_active=8, chunk=128).run(reqs)
    errs = {r.fid: r.error for r in rep.requests}
    assert errs[1] is not None and errs[0] is None and errs[2] is None
    assert rep.completed == 2


def test_fragment_batchable_limit_and_estimate():
    f = _frags(1, qubits=16, bond=64)[0]
    assert f.batchable()
    f.max_bond = 128
    assert not f.batchable()
    assert estimate_bytes(24, 64, 1000) > estimate_bytes(24, 32, 1000) > 0


def test_fragments_above_fused_limit_advance_in_their_own_group():
    frags = _frags(2, gates_per_update=(400,), n_updates=1, qubits=16, bond=128)
    frags += _frags(1, gates_per_update=(900,), n_updates=1)
    frags[2].fid = 2
    be = FakeBackend()
    reqs = [Request(i, i, 0, 0.0) for i in range(3)]
    rep = Server(frags, be, max_active=8, chunk=128, max_chunk=128).run(reqs)
    assert rep.completed == 3
    # every chunk call holds only fused-limit fragments (2) or only larger ones (0, 1)
    assert set(be.chunk_members) <= {(2,), (0, 1), (0,), (1,)}
    assert (2,) in be.chunk_members and (0, 1) in be.chunk_members
    for r in rep.requests:
        assert r.energy == pytest.approx(r.fid + 0.001 * frags[r.fid].updates[0][0].size)


def test_gradient_requests_served_between_chunks():
    frags = _frags(2, gates_per_update=(300,), n_updates=2)
    for f in frags:
        f.thetas = [np.full(3, 0.1 * (u + 1)) for u in range(2)]

    class GradBackend(FakeBackend):
        def gradient(self, frag, update):
            return float(frag.fid) + 0.5, np.asarray(frag.thetas[update]) * 2.0

    be = GradBackend()
    reqs = [Request(0, 0, 0, 0.0), Request(1, 1, 0, 0.0, kind="gradient"),
            Request(2, 0, 1, 0.0), Request(3, 1, 1, 0.0, kind="gradient")]
    rep = Server(frags, be, max_active=8, chunk=64).run(reqs)
    assert rep.completed == 4
    by = {r.rid: r for r in rep.requests}
    assert by[1].energy == 1.5 and np.allclose(by[1].gradient, 0.2)
    assert by[3].energy == 1.5 and np.allclose(by[3].gradient, 0.4)
    assert by[0].gradient is None and by[0].energy == pytest.approx(0.001 * 300)
    assert all(m == (0,) for m in be.chunk_members)  # gradient requests take no gate chunks
