"""Seeded synthetic inputs for the MPS-VQE energy evaluation.

This package builds the *inputs* of the energy evaluation and nothing else:
random molecular integrals, the Jordan-Wigner Pauli sum they define, gate
lists for the UCCSD and hardware-efficient ansatze, and the initial
Hartree-Fock bitstring.  It holds none of the matrix-product-state
arithmetic (gate contraction, SVD, canonical form, transfer matrices); both
the FP64 oracle and the HIP library consume what it produces.

Random numbers come from ``numpy.random.default_rng([230303681, config,
purpose])`` with purpose 0 = integrals, 1 = angles, 2 = string sample,
3 = arrivals, 4 = fragment shapes of the serving mix, so every workload is
reproducible from its config index.
"""

from .rng import workload_rng
from .hamiltonian import (
    PauliSum,
    random_integrals,
    jw_hamiltonian,
    sample_terms,
    hf_bits,
    generic_term_count,
)
from .circuits import (
    Gate,
    gate_h,
    gate_rx,
    gate_ry,
    gate_rz,
    gate_cnot,
    gate_swap,
    pauli_exponential_gates,
    uccsd_excitations,
    uccsd_exponentials,
    uccsd_gates,
    gsd_window_excitations,
    qubit_adapt_pool,
    brickwork_gates,
    fuse_gates,
    pack_gates,
)
from .configs import CONFIGS, build_config, build_serving_fragments

__all__ = [
    "workload_rng",
    "PauliSum",
    "random_integrals",
    "jw_hamiltonian",
    "sample_terms",
    "hf_bits",
    "generic_term_count",
    "Gate",
    "gate_h",
    "gate_rx",
    "gate_ry",
    "gate_rz",
    "gate_cnot",
    "gate_swap",
    "pauli_exponential_gates",
    "uccsd_excitations",
    "uccsd_exponentials",
    "gsd_window_excitations",
    "qubit_adapt_pool",
    "uccsd_gates",
    "brickwork_gates",
    "fuse_gates",
    "pack_gates",
    "CONFIGS",
    "build_config",
    "build_serving_fragments",
]
