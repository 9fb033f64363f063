"""GPU: mps_jacobi_svd_noalloc (device buffers in a fixed per-device scratch
array, no allocation) against mps_jacobi_svd (which allocates its
workspace) on the same inputs, two calls in a row with the second smaller:
a 512 x 512 complex matrix (the multi-launch register rounds) and then a
96 x 70 one (the one-workgroup kernel), so stale scratch contents from the
first call must not leak into the second.  Singular values are also checked
against LAPACK, and the size limit is an argument error."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rand(rng, n, m):
    return rng.normal(size=(n, m)) + 1j * rng.normal(size=(n, m))


@pytest.mark.parametrize("stream_kind", ["null", "torch"])
def test_noalloc_matches_allocating_entry(gpu_lib, stream_kind):
    import torch
    from paper_2303_03681_amd import binding
    stream = None if stream_kind == "null" else torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(4242)
    for n, m in ((512, 512), (96, 70), (7, 5)):
        print(f"noalloc Jacobi {n}x{m} ({stream_kind} stream)", flush=True)
        a = _rand(rng, n, m)
        s0, w0, k0 = binding.jacobi_svd(a)
        s1, w1, k1 = binding.jacobi_svd_noalloc(a, stream=stream)
        assert k1 == k0
        smax = s0[0]
        assert np.max(np.abs(s1 - s0)) <= 1e-12 * smax
        r = min(n, m)
        assert np.max(np.abs(w1[:r] - w0[:r])) <= 1e-10
        ref = np.linalg.svd(a, compute_uv=False)
        assert np.max(np.abs(s1[:r] - ref)) <= 1e-12 * smax
        # A = U diag(sigma) W with orthonormal W rows: |A W^+| column norms are sigma
        aw = a @ w1[:r].conj().T
        assert np.max(np.abs(np.linalg.norm(aw, axis=0) - s1[:r])) <= 1e-11 * smax
        assert np.all(np.abs(s1[r:]) <= 1e-12 * smax)  # surplus vectors converge to zero


def test_noalloc_limits(gpu_lib):
    from paper_2303_03681_amd import binding
    with pytest.raises(binding.MpsError) as err:
        binding.jacobi_svd_noalloc(np.ones((513, 4), complex))
    assert err.value.name == "MPS_ERR_ARG"
    with pytest.raises(binding.MpsError) as err:
        binding.jacobi_svd_noalloc(np.ones((4, 513), complex))
    assert err.value.name == "MPS_ERR_ARG"
