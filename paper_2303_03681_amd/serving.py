"""Continuous-batching request loop for VQE energy requests on resident MPSs.

A fragment is one small molecule-sized problem (qubits, bond dimension,
Hamiltonian plan, a list of parameter updates each compiled to a gate list).
A request asks for the energy of one fragment at one update; updates of one
fragment are served in order (an update may start only after the previous
one of the same fragment has finished).  Each fragment's MPS stays resident
on the device between its updates, together with its cached environment
setup, until memory is needed for another fragment.

The loop (Server.run):
  1. admit arrived requests while a slot is free and the fragment fits in the
     device-memory budget (idle resident fragments are evicted, least recently
     used first, to make room); an admitted request resets its MPS to the
     Hartree-Fock product state;
  2. advance every admitted request by one chunk of gates, in two batched
     calls (mps_apply_gates_multi) that run side by side: fragments whose
     bonds are within the fused limit (capacity <= 64) take one device
     launch per gate index, one workgroup per request; larger fragments take
     batched steps, the step's gates of all of them in one multi-workgroup
     SVD batch; either way all dependent gate chains move together;
  3. requests whose gates are done get their energy (the Pauli-sum
     expectation from the boundary environments, divided by <psi|psi>; no
     canonicalisation sweep) between chunks, all of an iteration's finished
     requests in one pass whose launches they share
     (mps_expect_pauli_sum_multi); gradient-step requests (energy and
     parameter-shift dE/dtheta of the fragment's UCCSD at the update's
     angles) are also served between chunks;
  4. finished requests free their slot; arrivals are admitted between chunks.

Energies run between gate chunks rather than beside them: the expectation
path synchronises with the host many times, and streams
beyond the device's few hardware queues share a queue in submission order, so
each of those waits could otherwise stall behind a whole gate chunk.  Chunks
are sized (per group) to a target duration so that arrivals wait at most
about that long to join.

Latency of a request is arrival -> energy available; the report gives p50 and
p99 next to the throughput.  The energy of a request does not depend on what
else is in flight: each request's arithmetic is the same sequence of kernels
on its own data.

The policy is separated from the device through a small backend interface so
that scheduling can be tested on the CPU.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np


@dataclass
class Fragment:
    fid: int
    n_qubits: int
    max_bond: int
    cutoff: float
    bits: np.ndarray
    codes: np.ndarray                 # Pauli strings, n_terms x n_qubits
    coeffs: np.ndarray
    updates: list                     # per update: (q0, q1, u_packed)
    est_bytes: int = 0                # device-memory estimate before first use
    thetas: list | None = None        # per update: the UCCSD angles (gradient requests)
    n_electrons: int = 0
    window: int | None = None

    @property
    def n_terms(self) -> int:
        return int(self.coeffs.size)

    @classmethod
    def from_dict(cls, d: dict) -> "Fragment":
        return cls(d["fid"], d["n_qubits"], d["max_bond"], d["cutoff"], d["bits"], d["codes"],
                   d["coeffs"], d["updates"], thetas=d.get("thetas"), n_electrons=d.get("n_electrons", 0),
                   window=d.get("window"))

    def batchable(self) -> bool:
        """Every bond capacity <= 64: its gates run on the fused one-workgroup
        path (else on batched multi-workgroup steps shared with the other
        large fragments)."""
        return max(min(self.max_bond, 2 ** min(b, self.n_qubits - b))
                   for b in range(self.n_qubits + 1)) <= 64


@dataclass
class Request:
    rid: int
    fid: int
    update: int
    arrival: float                    # seconds after the start of the run
    admitted: float = math.nan
    gates_done: float = math.nan
    finish: float = math.nan
    energy: float = math.nan
    error: str | None = None
    kind: str = "energy"              # "energy" | "gradient" (energy and dE/dtheta)
    gradient: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def estimate_bytes(n_qubits: int, max_bond: int, n_env_updates: int, prec_bytes: int = 8) -> int:
    """Upper estimate of one fragment's device memory: two site and lambda
    buffers, the gate workspaces, the environment pool and its scratch."""
    caps = [min(max_bond, 2 ** min(b, n_qubits - b)) for b in range(n_qubits + 1)]
    sites = sum(2 * 2 * caps[q] * caps[q + 1] * 16 for q in range(n_qubits))
    dmax = max(caps)
    ws = 2 * (2 * dmax) ** 2 * 16 + 2 * dmax * dmax * 16
    pool = (n_env_updates + 2 * (n_qubits + 1)) * dmax * dmax * prec_bytes
    prepared = 2 * sites
    scratch = 64 * dmax * 2 * dmax * prec_bytes
    return int(sites + ws + pool + prepared + scratch + (8 << 20))


# --------------------------------------------------------------------------
# backends


class GpuBackend:
    """The HIP library: one Mps handle per resident fragment; batched gate
    chunks on one server stream; energies on the handles' own streams."""

    def __init__(self, prec: str = "c64"):
        import torch

        from . import binding
        self.binding = binding
        self.prec = prec
        self.stream = torch.cuda.Stream()
        self.plans: dict[int, object] = {}
        self.grads: dict[int, object] = {}

    def _plan(self, frag: Fragment):
        if frag.fid not in self.plans:
            self.plans[frag.fid] = self.binding.PauliSum(frag.codes, frag.coeffs)
        return self.plans[frag.fid]

    def create(self, frag: Fragment):
        self._plan(frag)
        return self.binding.Mps(frag.n_qubits, frag.max_bond, frag.cutoff, bits=frag.bits)

    def plan_updates(self, frag: Fragment) -> int:
        st = self._plan(frag).stats()
        return int(st["left_updates"] + st["right_updates"])

    def reset(self, handle, frag: Fragment):
        handle.reset(frag.bits)

    def apply_chunk(self, items):
        """items: list of (handle, q0, q1, u) slices; returns gates applied."""
        return self.binding.apply_gates_multi([it[0] for it in items],
                                              [(it[1], it[2], it[3]) for it in items],
                                              stream=self.stream.cuda_stream)

    def expect(self, handle, frag: Fragment) -> float:
        return handle.expect(self._plan(frag), self.prec)

    def expect_many(self, pairs):
        """Energies of several (handle, fragment) pairs in one pass: their
        environment updates of equal depth share launches."""
        return list(self.binding.expect_multi([h for h, _ in pairs], [self._plan(f) for _, f in pairs],
                                              self.prec))

    def gradient(self, frag: Fragment, update: int):
        """Energy and parameter-shift gradient of the fragment's UCCSD at the
        update's angles (f1); the gradient engine and its handles are kept
        per fragment."""
        from .gradients import UccsdGradient
        if frag.thetas is None:
            raise ValueError(f"fragment {frag.fid} carries no UCCSD angles")
        g = self.grads.get(frag.fid)
        if g is None:
            g = UccsdGradient(frag.n_qubits, frag.n_electrons, self._plan(frag), frag.max_bond,
                              frag.cutoff, bits=frag.bits, window=frag.window, prec=self.prec)
            self.grads[frag.fid] = g
        return g.energy_and_gradient(frag.thetas[update])

    def device_bytes(self, handle) -> int:
        return int(handle.device_bytes())

    def destroy(self, handle):
        handle.close()

    def shutdown(self):
        for g in self.grads.values():
            g.close()
        self.grads.clear()


# --------------------------------------------------------------------------
# the request loop


@dataclass
class _Active:
    req: Request
    frag: Fragment
    handle: object
    cursor: int = 0


@dataclass
class ServeReport:
    requests: list
    span_s: float
    completed: int
    strings: int
    max_active: int
    mean_active: float
    evictions: int
    chunks: int

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.requests if not math.isnan(r.finish)]) * 1e3
        out = {
            "completed": self.completed,
            "span_s": self.span_s,
            "requests_per_s": self.completed / self.span_s if self.span_s > 0 else 0.0,
            "strings_per_s": self.strings / self.span_s if self.span_s > 0 else 0.0,
            "max_active": self.max_active,
            "mean_active": self.mean_active,
            "evictions": self.evictions,
            "gate_chunks": self.chunks,
        }
        if lat.size:
            out["latency_ms"] = {"p50": float(np.percentile(lat, 50)),
                                 "p99": float(np.percentile(lat, 99)),
                                 "mean": float(lat.mean()), "max": float(lat.max())}
        return out


class Server:
    def __init__(self, fragments: list[Fragment], backend, max_active: int = 64,
                 hbm_budget: int | None = None, chunk: int = 256, chunk_s: float = 0.5,
                 max_chunk: int = 4096, clock=time.perf_counter, sleep=time.sleep, log=None):
        self.frags = {f.fid: f for f in fragments}
        self.backend = backend
        self.max_active = max_active
        self.budget = hbm_budget
        self.chunk = chunk
        self.chunk_s = chunk_s
        self.max_chunk = max_chunk
        self.log = log
        self.clock = clock
        self.sleep = sleep
        self.resident: dict[int, object] = {}      # fid -> handle
        self.resident_bytes: dict[int, int] = {}
        self.last_used: dict[int, float] = {}
        self.busy: set[int] = set()                # fragments with a request in flight
        self.evictions = 0
        self.chunks = 0

    # memory accounting -------------------------------------------------
    def _need(self, frag: Fragment) -> int:
        if frag.fid in self.resident:
            return 0
        if not frag.est_bytes:
            frag.est_bytes = estimate_bytes(frag.n_qubits, frag.max_bond,
                                            self.backend.plan_updates(frag))
        return frag.est_bytes

    def _used(self) -> int:
        return sum(self.resident_bytes.values())

    def _make_room(self, need: int) -> bool:
        if self.budget is None:
            return True
        while self._used() + need > self.budget:
            idle = [f for f in self.resident if f not in self.busy]
            if not idle:
                return False
            victim = min(idle, key=lambda f: self.last_used.get(f, 0.0))
            self.backend.destroy(self.resident.pop(victim))
            self.resident_bytes.pop(victim, None)
            self.evictions += 1
        return True

    # the loop ----------------------------------------------------------
    def run(self, requests: list[Request], timeout_s: float = 3600.0) -> ServeReport:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        per_frag: dict[int, list[int]] = {}
        for r in reqs:
            if r.fid not in self.frags:
                raise ValueError(f"request {r.rid}: unknown fragment {r.fid}")
            if not 0 <= r.update < len(self.frags[r.fid].updates):
                raise ValueError(f"request {r.rid}: fragment {r.fid} has no update {r.update}")
            per_frag.setdefault(r.fid, []).append(r.update)
        for fid, ups in per_frag.items():
            if sorted(ups) != list(range(len(ups))):
                raise ValueError(f"fragment {fid}: requested updates must be 0, 1, ... once each")
        next_update = {fid: 0 for fid in self.frags}  # updates are served in order
        waiting: list[Request] = []                    # arrived, not admitted
        upcoming = list(reqs)
        active: list[_Active] = []                     # gate chains in progress
        ready: list[_Active] = []                      # gates done, energy pending
        grads: list[_Active] = []                      # gradient requests (served between chunks)
        done: list[Request] = []
        t0 = self.clock()
        active_samples = []
        max_seen = 0
        strings = 0
        steps = {True: self.chunk, False: self.chunk}  # chunk length per group (fused / batched)

        def finish(a: _Active, energy=None, error=None):
            nonlocal strings
            if error is None:
                a.req.energy = float(energy)
                strings += a.frag.n_terms
            else:
                a.req.error = error
            a.req.finish = self.clock() - t0
            self.resident_bytes[a.req.fid] = max(self.resident_bytes.get(a.req.fid, 0),
                                                 self.backend.device_bytes(a.handle))
            self._release(a, next_update)
            done.append(a.req)

        while len(done) < len(reqs):
            now = self.clock() - t0
            if now > timeout_s:
                raise TimeoutError("serving loop exceeded its time limit")
            while upcoming and upcoming[0].arrival <= now:
                waiting.append(upcoming.pop(0))
            # 1. admission (arrival order; a request waits for its fragment's
            #    previous update and for a slot and memory)
            in_flight = len(active) + len(ready) + len(grads)
            idle_before = in_flight == 0
            still = []
            for r in waiting:
                frag = self.frags[r.fid]
                if (in_flight >= self.max_active or r.fid in self.busy
                        or r.update != next_update[r.fid]):
                    still.append(r)
                    continue
                need = self._need(frag)
                if not self._make_room(need):
                    still.append(r)
                    continue
                if r.fid not in self.resident:
                    self.resident[r.fid] = self.backend.create(frag)
                    self.resident_bytes[r.fid] = need
                h = self.resident[r.fid]
                self.backend.reset(h, frag)
                r.admitted = self.clock() - t0
                self.busy.add(r.fid)
                (grads if r.kind == "gradient" else active).append(_Active(r, frag, h))
                in_flight += 1
            # nothing was in flight and nothing could be admitted: no later
            # completion can free memory, so the budget is too small
            stuck = idle_before and in_flight == 0 and bool(waiting) and all(
                r.update == next_update[r.fid] and r.fid not in self.busy for r in waiting[:1])
            waiting = still
            max_seen = max(max_seen, in_flight)
            # 2. energies of requests whose gates are done (together, when the
            #    backend can share their launches); gradient requests
            many = getattr(self.backend, "expect_many", None)
            if many is not None and len(ready) > 1:
                try:
                    for a, e in zip(ready, many([(a.handle, a.frag) for a in ready])):
                        finish(a, e)
                    ready = []
                except Exception:
                    pass  # one at a time below, so that an error names its request
            for a in ready:
                try:
                    finish(a, self.backend.expect(a.handle, a.frag))
                except Exception as err:
                    finish(a, error=str(err))
            ready = []
            for a in grads:
                try:
                    e, g = self.backend.gradient(a.frag, a.req.update)
                    a.req.gradient = np.asarray(g)
                    a.req.gates_done = self.clock() - t0
                    finish(a, e)
                except Exception as err:
                    finish(a, error=str(err))
            grads = []
            # 3. one gate chunk for every admitted request: fragments within the
            #    fused limit advance together on one-workgroup launches, larger
            #    ones together on batched multi-workgroup steps; the two groups'
            #    calls run side by side (the library releases the interpreter)
            if active:
                groups = {}
                for a in active:
                    groups.setdefault(a.frag.batchable(), []).append(a)
                active_samples.append(len(active))

                def run_group(small, members):
                    items = []
                    for a in members:
                        q0, q1, u = a.frag.updates[a.req.update]
                        c1 = min(len(q0), a.cursor + steps[small])
                        items.append((a.handle, q0[a.cursor:c1], q1[a.cursor:c1], u[a.cursor:c1]))
                    tc = self.clock()
                    failed = None
                    try:
                        applied = self.backend.apply_chunk(items)
                    except Exception as err:  # a failed gate: only its request fails
                        applied = getattr(err, "n_done", None)
                        failed = err
                        if applied is None:
                            raise
                    return items, applied, failed, self.clock() - tc

                if len(groups) > 1:
                    from concurrent.futures import ThreadPoolExecutor
                    with ThreadPoolExecutor(max_workers=2) as pool:
                        futs = {k: pool.submit(run_group, k, v) for k, v in groups.items()}
                        results = {k: f.result() for k, f in futs.items()}
                else:
                    results = {k: run_group(k, v) for k, v in groups.items()}
                keep = []
                for small, members in groups.items():
                    items, applied, failed, dt = results[small]
                    self.chunks += 1
                    longest = max(len(it[1]) for it in items)
                    if longest > 0 and dt > 0:  # size the group's next chunk to the target duration,
                        # growing at most 2x a chunk (early gates, on small bonds, are far cheaper)
                        want = min(self.chunk_s * longest / dt, 2 * longest)
                        steps[small] = int(min(self.max_chunk, max(16, want)))
                    for a, it, k in zip(members, items, applied):
                        n_slice = len(it[1])
                        if k < n_slice:  # this request's gate failed
                            finish(a, error=str(failed))
                            continue
                        a.cursor += n_slice
                        if a.cursor >= len(a.frag.updates[a.req.update][0]):
                            a.req.gates_done = self.clock() - t0
                            ready.append(a)
                        else:
                            keep.append(a)
                    if self.log:
                        self.log(f"chunk {self.chunks} ({'fused' if small else 'batched'}): {len(items)} "
                                 f"chains x {longest} gates in {dt:.2f} s; {len(done)}/{len(reqs)} done")
                active = keep
            # 4. idle: wait for the next arrival
            if not active and not ready and not grads:
                if stuck:
                    r = waiting[0]
                    raise RuntimeError(f"request {r.rid} (fragment {r.fid}) cannot be admitted: "
                                       f"needs {self._need(self.frags[r.fid])} bytes, "
                                       f"budget {self.budget}")
                if upcoming and not waiting:
                    self.sleep(max(0.0, min(0.05, upcoming[0].arrival - (self.clock() - t0))))
        span = max(r.finish for r in done) - min(r.arrival for r in done)
        return ServeReport(done, span, sum(1 for r in done if r.error is None), strings, max_seen,
                           float(np.mean(active_samples)) if active_samples else 0.0,
                           self.evictions, self.chunks)

    def _release(self, a: _Active, next_update):
        self.busy.discard(a.req.fid)
        next_update[a.req.fid] = a.req.update + 1
        self.last_used[a.req.fid] = self.clock()

    def close(self):
        for h in self.resident.values():
            self.backend.destroy(h)
        self.resident.clear()
        self.resident_bytes.clear()


# --------------------------------------------------------------------------
# workload: DMET-like fragments with windowed UCCSD circuits


def poisson_arrivals(n: int, rate: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def make_requests(n_fragments: int, n_updates: int, rate: float, rng) -> list[Request]:
    """Request r goes to fragment r mod n_fragments, update r // n_fragments."""
    t = poisson_arrivals(n_fragments * n_updates, rate, rng)
    return [Request(r, r % n_fragments, r // n_fragments, float(t[r]))
            for r in range(n_fragments * n_updates)]
