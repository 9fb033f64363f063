"""The five synthetic workloads of the energy-evaluation benchmark.

C1  8 qubits (4 orbitals, 4 electrons), UCCSD, D <= 16 (no truncation)
C2  24 qubits (12 orbitals, 12 electrons), UCCSD, D = 64, cutoff 1e-10
C3  50 qubits (25 orbitals, 24 electrons), brickwork 20 layers, D = 256,
    2^18 strings sampled from the JW expansion
C4  serving mix of DMET-like fragments (12 .. 40 qubits, D in {32, 64, 128})
C5  100 qubits, brickwork 40 layers, D = 512, 2^20 sampled strings

The paper's molecules (H2, hydrogen chains, ethane, DMET fragments of
protein-ligand complexes) are not available; seeded random integrals with the
symmetry of real ones stand in for them.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .circuits import Gate, brickwork_gates, fuse_gates, pack_gates, uccsd_gates, uccsd_n_params
from .hamiltonian import PauliSum, hf_bits, jw_hamiltonian, random_integrals, sample_terms
from .rng import PURPOSE_ANGLES, PURPOSE_INTEGRALS, PURPOSE_MIX, PURPOSE_SAMPLE, workload_rng


@dataclass
class ConfigSpec:
    index: int
    name: str
    n_spatial: int
    n_electrons: int
    ansatz: str  # "uccsd" | "brickwork"
    max_bond: int
    cutoff: float
    layers: int = 0
    n_strings: int = 0  # 0 = full expansion
    angle_range: float = 0.1


CONFIGS = {
    1: ConfigSpec(1, "8q-uccsd-D16", 4, 4, "uccsd", 16, 1e-14, angle_range=0.1),
    2: ConfigSpec(2, "24q-uccsd-D64", 12, 12, "uccsd", 64, 1e-10, angle_range=0.1),
    3: ConfigSpec(3, "50q-brickwork20-D256", 25, 24, "brickwork", 256, 1e-14, layers=20,
                  n_strings=1 << 18, angle_range=np.pi),
    5: ConfigSpec(5, "100q-brickwork40-D512", 50, 50, "brickwork", 512, 1e-14, layers=40,
                  n_strings=1 << 20, angle_range=np.pi),
}


@dataclass
class Workload:
    spec: ConfigSpec
    n_qubits: int
    bits: np.ndarray
    gates: list
    psum: PauliSum
    h: np.ndarray = field(repr=False)
    g: np.ndarray = field(repr=False)
    full_terms: int = 0


def build_config(index: int, fuse: bool = True, with_gates: bool = True,
                 n_spatial: int | None = None, layers: int | None = None,
                 n_strings: int | None = None, progress=None) -> Workload:
    """Deterministic workload for config ``index``; the keyword overrides
    shrink it (same recipe, smaller sizes) for tests."""
    spec = CONFIGS[index]
    n_s = n_spatial if n_spatial is not None else spec.n_spatial
    n_q = 2 * n_s
    n_e = min(spec.n_electrons, n_q) if n_spatial is None else min(spec.n_electrons, n_q - 2)
    h, g = random_integrals(n_s, workload_rng(index, PURPOSE_INTEGRALS))
    full = jw_hamiltonian(h, g, progress=progress)
    ns = spec.n_strings if n_strings is None else n_strings
    psum = sample_terms(full, ns, workload_rng(index, PURPOSE_SAMPLE)) if ns else full
    bits = hf_bits(n_q, n_e)
    gates: list[Gate] = []
    if with_gates:
        rng = workload_rng(index, PURPOSE_ANGLES)
        if spec.ansatz == "uccsd":
            theta = rng.uniform(-spec.angle_range, spec.angle_range,
                                size=uccsd_n_params(n_q, n_e))
            gates = uccsd_gates(n_q, n_e, theta)
        else:
            L = spec.layers if layers is None else layers
            angles = rng.uniform(-spec.angle_range, spec.angle_range, size=(L, n_q, 2))
            gates = brickwork_gates(n_q, angles)
        if fuse:
            gates = fuse_gates(gates, n_q)
    return Workload(spec, n_q, bits, gates, psum, h, g, full.n_terms)


def build_serving_fragments(n_fragments: int, n_updates: int,
                            qubits=(12, 16, 20, 24, 28, 32, 36, 40), bonds=(32, 64, 128),
                            max_strings: int = 1 << 16, window: int = 5,
                            cutoff: float = 1e-10) -> list[dict]:
    """DMET-like fragments of the serving mix (config 4): qubit count and bond
    dimension drawn uniformly from the given sets, N_e = n/2, each with its
    own random integrals, its JW sum sampled to at most max_strings, and
    n_updates pre-drawn angle vectors U(-0.1, 0.1) of the windowed UCCSD
    ansatz, each compiled (fused, packed) to a gate list."""
    mix = workload_rng(4, PURPOSE_MIX)
    shapes = [(int(mix.choice(qubits)), int(mix.choice(bonds))) for _ in range(n_fragments)]
    out = []
    for fid, (n, D) in enumerate(shapes):
        ne = n // 2
        h, g = random_integrals(n // 2, workload_rng(4, PURPOSE_INTEGRALS, fid + 1))
        full = jw_hamiltonian(h, g)
        psum = sample_terms(full, max_strings, workload_rng(4, PURPOSE_SAMPLE, fid + 1))
        npar = uccsd_n_params(n, ne, window=window)
        thetas = workload_rng(4, PURPOSE_ANGLES, fid + 1).uniform(-0.1, 0.1, size=(n_updates, npar))
        updates = [pack_gates(fuse_gates(uccsd_gates(n, ne, th, window=window), n)) for th in thetas]
        out.append({"fid": fid, "n_qubits": n, "max_bond": D, "cutoff": cutoff,
                    "bits": hf_bits(n, ne), "codes": psum.codes, "coeffs": psum.coeffs,
                    "updates": updates, "full_terms": full.n_terms,
                    "thetas": [np.array(t) for t in thetas], "n_electrons": ne, "window": window})
    return out
