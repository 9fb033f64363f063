"""Test helper: the oracle's two-qubit update of two exported sites, for
checking a truncation the GPU took along its own trajectory (Eqs. C, C~,
svd, Bl with the oracle's LAPACK SVD)."""

import numpy as np


def oracle_gate(b0, b1, lam_l, u, D, cutoff):
    """Sites (b0, b1) with left lambda lam_l under the 4x4 gate u: the kept
    normalised singular values, the gate's discarded weight and the full
    spectrum."""
    from oracle import MpsOracle
    spec = {}

    class Spy(MpsOracle):
        def _svd(self, mat):
            out = super()._svd(mat)
            spec["s"] = out[1]
            return out

    o = Spy(2, D, cutoff)
    o.B = [b0, b1]
    o.lam = [np.asarray(lam_l, float), np.ones(b0.shape[2]), np.ones(1)]
    o.apply_2q(0, u)
    return o.lam[1], o.discarded, spec["s"]


def check_gate(m, g, q0, q1, u, D, cutoff):
    """Apply two-qubit gate g (packed arrays q0, q1, u) alone to the GPU state
    m and redo it in the oracle on the exported sites.  Asserts equal bond
    dimensions; returns (max |d lambda|, |d w|, kept rank, oracle spectrum,
    the oracle's discarded weight of the gate)."""
    q = int(q0[g])
    assert int(q1[g]) == q + 1
    b0, lam_l = m.export_site(q)
    b1, _ = m.export_site(q + 1)
    d0 = m.discarded_weight()
    assert m.apply_gates(q0[g:g + 1], q1[g:g + 1], u[g:g + 1]) == 1
    _, lam_new = m.export_site(q + 1)
    dw = m.discarded_weight() - d0
    umat = (u[g, :, 0] + 1j * u[g, :, 1]).reshape(4, 4)
    lam_ref, dw_ref, s = oracle_gate(b0, b1, lam_l, umat, D, cutoff)
    assert lam_new.size == lam_ref.size, (g, q, lam_new.size, lam_ref.size)
    return float(np.max(np.abs(lam_new - lam_ref))), abs(dw - dw_ref), lam_ref.size, s, dw_ref
