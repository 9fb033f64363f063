"""Writes c2_windowed_24q.json: FP64 oracle results for the 24-qubit workload
(12 orbitals, 12 electrons, full random-integral JW sum of 29,737 strings)
under the windowed UCCSD circuit (excitations within 5 consecutive orbitals,
angles U(-0.1, 0.1)), SVD cutoff 1e-10, at D = 64 (the workload's bond
dimension), D = 128 (both cut at the bond cap, at near-degenerate singular
values among others) and D = 256 (the state never reaches the cap: threshold
cuts only).

Test infrastructure: calls only oracle/ and workloads/.  Run from the
repository root:  python tests/golden/make_c2_windowed.py
"""

import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import MpsOracle  # noqa: E402
from workloads import build_config, fuse_gates, workload_rng  # noqa: E402
from workloads.circuits import uccsd_gates, uccsd_n_params  # noqa: E402


def c2_windowed_gates():
    w = build_config(2, with_gates=False)
    n, ne = w.n_qubits, 12
    th = workload_rng(2, 1).uniform(-0.1, 0.1, uccsd_n_params(n, ne, window=5))
    return w, fuse_gates(uccsd_gates(n, ne, th, window=5), n)


def main():
    w, gates = c2_windowed_gates()
    out = {"workload": "24q (12 orbitals, 12 e-), full JW sum, windowed UCCSD (window 5), "
                       "angles U(-0.1, 0.1) from workload_rng(2, 1), cutoff 1e-10",
           "n_gates": len(gates), "n_terms": int(w.psum.n_terms), "cases": {}}
    sample = np.arange(0, w.psum.n_terms, 97)
    for D in (64, 128, 256):
        o = MpsOracle(w.n_qubits, D, 1e-10, w.bits)
        o.apply_gates(gates)
        dims = o.bond_dims()
        disc = o.discarded
        o.canonicalize()
        per = o.expect_terms(w.psum.codes).real
        out["cases"][str(D)] = {
            "bond_dims": [int(d) for d in dims],
            "discarded_weight": float(disc),
            "energy": math.fsum(w.psum.coeffs * per),
            "sample_terms": sample.tolist(),
            "sample_values": per[sample].tolist(),
        }
        print(f"D={D}: E={out['cases'][str(D)]['energy']:.12f} dims={dims} disc={disc:.3e}", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_windowed_24q.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
