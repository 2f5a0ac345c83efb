"""The inversion entry point that allocates nothing (bem_dense_invert_noalloc: the library's fixed
device workspace) against the allocating one (bem_dense_invert) through the C ABI: two calls in a
row, the second smaller, each compared with the allocating call on the same matrix (same kernels:
bitwise equal inverses and health) and with LAPACK; sizes beyond the workspace are refused."""
from __future__ import annotations

import numpy as np
import pytest

import paper_2106_06184_amd as B

pytestmark = pytest.mark.gpu


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return A + (2.0 - 0.7j) * np.eye(n)


def test_noalloc_inverse_equals_allocating_inverse():
    import torch
    ctx = B.bem_create(0)
    try:
        for n, ld, seed in [(1500, 1504, 1), (333, 333, 2)]:  # the second call is smaller
            print(f"no-alloc inversion: n {n}, ld {ld}, seed {seed}", flush=True)
            A = np.zeros((n, ld), np.complex128)
            A[:, :n] = _matrix(n, seed)
            d1 = torch.tensor(A, device="cuda")
            d2 = torch.tensor(A, device="cuda")
            rc1, h1 = B.bem_dense_invert_noalloc(ctx, d1.data_ptr(), n, ld)
            rc2, h2 = B.bem_dense_invert(ctx, d2.data_ptr(), n, ld)
            torch.cuda.synchronize()
            assert rc1 == B.BEM_OK and rc2 == B.BEM_OK
            got, want = d1.cpu().numpy()[:, :n], d2.cpu().numpy()[:, :n]
            assert np.array_equal(got, want)
            assert h1 == h2
            ref = np.linalg.inv(A[:, :n])
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            print(f"  rel err vs LAPACK {err:.2e}, pivot ratio {h1[0]:.2e}, probe {h1[1]:.2e}", flush=True)
            assert err < 1e-13 and h1[1] < 1e-13
        big = torch.zeros((2049, 2049), dtype=torch.complex128, device="cuda")
        with pytest.raises(B.BemError, match="2048"):
            B.bem_dense_invert_noalloc(ctx, big.data_ptr(), 2049, 2049)
    finally:
        B.bem_destroy(ctx)
