"""GPU: the split-16-bit environment GEMMs on bond dimensions that are not
multiples of eight.  A thread stages eight consecutive K values of a chunk;
in the second half of the transfer-matrix update (K runs over the physical
index s and the left bond) eight values of a chunk can then straddle the two
s blocks and are fetched one by one, while the other chunks of the same
full 64 x 64 tile take the eight-value fetch with the conjugation and the
Pauli phase applied to whole split planes.  A random right-canonical
16-qubit MPS with bonds up to 100 is imported, its expectations are taken
from the boundary environments (Eqs. expec1, expec2 divided by <psi|psi>),
and every string in every precision is compared with the dense statevector
of the same tensors."""

import numpy as np
import pytest

from oracle import dense_expect_pauli

pytestmark = pytest.mark.gpu

N = 16
BONDS = [1, 2, 4, 8, 16, 32, 64, 100, 100, 100, 64, 32, 16, 8, 4, 2, 1]


def _say(msg):
    print(msg, flush=True)


def _right_canonical_sites(rng):
    """B_q[s][a][b] with sum_s B^s B^s+ = I (orthonormal rows of the
    D_q x 2 D_{q+1} matrix [B^0 | B^1])."""
    sites = []
    for q in range(N):
        dl, dr = BONDS[q], BONDS[q + 1]
        z = rng.normal(size=(2 * dr, dl)) + 1j * rng.normal(size=(2 * dr, dl))
        qm, _ = np.linalg.qr(z)  # 2 dr x dl, orthonormal columns
        rows = qm.conj().T       # dl x 2 dr, orthonormal rows
        sites.append(np.stack([rows[:, :dr], rows[:, dr:]]))
    return sites


def _dense(sites):
    psi = np.ones((1, 1), dtype=complex)
    for b in sites:
        psi = np.einsum("pa,sab->psb", psi, b).reshape(-1, b.shape[2])
    return psi.reshape((2,) * N)


def test_split_environments_on_bonds_not_multiple_of_eight(gpu_lib):
    from paper_2303_03681_amd import binding
    rng = np.random.default_rng(2303)
    sites = _right_canonical_sites(rng)
    psi = _dense(sites)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    m = binding.Mps(N, 128, 1e-14)
    for q, b in enumerate(sites):
        m.import_site(q, b, np.full(BONDS[q], BONDS[q] ** -0.5))
    m.apply_gate(0, -1, np.eye(2))  # not canonical any more: boundary environments
    assert list(m.bond_dims()) == BONDS
    codes = rng.integers(0, 4, size=(600, N)).astype(np.uint8)
    codes[:200, 5:11] = rng.integers(1, 4, size=(200, 6))  # letters on the 100-wide bonds
    ref = np.array([dense_expect_pauli(psi, c).real for c in codes])
    plan = binding.PauliSum(codes, rng.normal(size=len(codes)))
    # measured: c128 4e-17, c64 1.1e-8, split-F16 6.8e-9, split-BF16 3.3e-7
    for prec, tol in (("c128", 1e-12), ("c64", 1e-6), ("split_f16", 1e-7), ("split_bf16", 5e-6)):
        _, per = m.expect(plan, prec, per_term=True)
        err = float(np.max(np.abs(per - ref)))
        _say(f"  {prec}: max |<P> - dense| {err:.2e}")
        assert err < tol, (prec, err)
    m.close()
    plan.close()
