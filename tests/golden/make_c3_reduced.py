"""Writes c3_reduced.json: FP64 oracle results for two reduced cases of the
50-qubit brickwork workload's recipe (random-integral JW Hamiltonian sampled
uniformly, hardware-efficient brickwork ansatz with Ry/Rz folded into the
CNOTs, angles U(-pi, pi), cutoff 1e-14), sized so that the GPU runs them
through the same code paths as the full 50-qubit evaluation:

  36q_D256: 18 orbitals (36 qubits), 12 layers, D = 256, 4096 strings.
            The later sub-layers hold 9-10 gates whose two-site matrix is
            512 x 512 (the multi-item register Jacobi rounds, split over
            item groups above 256 workgroups per round), the environment
            products of saturated D = 256 bonds, and the closing traces.
  28q_D512: 14 orbitals (28 qubits), 13 layers, D = 512, 512 strings.
            Gates whose two-site matrix is 1024 x 1024 (the wide-row Jacobi
            rounds, 4-5 items per sub-layer) and the D = 512 products of
            Eqs. (C) and (Bl).

For every truncation at the bond cap the relative gap
(sigma_k - sigma_{k+1}) / sigma_1 is recorded: the kept subspace is fixed to
about 1e-16 / gap, so a smallest gap far above 1e-12 makes bond dimensions,
discarded weight, strings and energy exact-parity quantities (the SVD's
rounding does not choose between truncations).

Test infrastructure: calls only oracle/ and workloads/.  Run from the
repository root:  python tests/golden/make_c3_reduced.py
"""

import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import MpsOracle  # noqa: E402
from workloads import build_config  # noqa: E402

CASES = {
    "36q_D256": {"n_spatial": 18, "layers": 12, "max_bond": 256, "n_strings": 4096},
    "28q_D512": {"n_spatial": 14, "layers": 13, "max_bond": 512, "n_strings": 512},
}


class GapOracle(MpsOracle):
    """The oracle MPS, recording the relative gap at every cut at the cap."""

    def __init__(self, *a, **k):
        self.cap_gaps = []
        super().__init__(*a, **k)

    def _svd(self, m):
        u, s, vh = super()._svd(m)
        if s.size > self.max_bond and s[self.max_bond] > self.cutoff * math.sqrt(float(np.sum(s * s))):
            self.cap_gaps.append(float((s[self.max_bond - 1] - s[self.max_bond]) / s[0]))
        return u, s, vh


def run_case(name, spec):
    t0 = time.time()
    w = build_config(3, n_spatial=spec["n_spatial"], layers=spec["layers"], n_strings=spec["n_strings"])
    o = GapOracle(w.n_qubits, spec["max_bond"], w.spec.cutoff, w.bits)
    o.apply_gates(w.gates)
    dims = o.bond_dims()
    disc = o.discarded
    print(f"{name}: {len(w.gates)} gates in {time.time() - t0:.0f} s, max bond {max(dims)}, "
          f"{len(o.cap_gaps)} cap cuts, smallest gap {min(o.cap_gaps):.2e}", flush=True)
    o.canonicalize()
    per = o.expect_terms(w.psum.codes).real
    e = math.fsum(w.psum.coeffs * per)
    print(f"{name}: E = {e:.15f}, discarded {disc:.6e}, {time.time() - t0:.0f} s", flush=True)
    return {
        "recipe": (f"config-3 recipe at {spec['n_spatial']} orbitals ({w.n_qubits} qubits), "
                   f"{spec['layers']} brickwork layers, D = {spec['max_bond']}, "
                   f"{spec['n_strings']} sampled strings, cutoff {w.spec.cutoff}"),
        **spec,
        "n_qubits": w.n_qubits,
        "n_gates": len(w.gates),
        "n_terms": int(w.psum.n_terms),
        "bond_dims": [int(d) for d in dims],
        "discarded_weight": float(disc),
        "cap_cuts": len(o.cap_gaps),
        "min_cap_gap": min(o.cap_gaps),
        "energy": e,
        "values": per.tolist(),
    }


def main():
    out = {name: run_case(name, spec) for name, spec in CASES.items()}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_reduced.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
