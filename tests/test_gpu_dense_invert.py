"""Device dense inversion (blocked Gauss-Jordan without pivoting) through the C ABI: accuracy on
well-posed matrices, and loud failure (BEM_E_NUMERIC) where elimination without pivoting breaks
down - a zero or tiny leading pivot, a singular matrix, a non-finite entry.  The references are
numpy's LAPACK inverse and the matrices' own construction."""
from __future__ import annotations

import numpy as np
import pytest

import paper_2106_06184_amd as B

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.fixture(scope="module")
def ctx():
    c = B.bem_create(0)
    yield c
    B.bem_destroy(c)


def _invert(torch, ctx, A, ld=None):
    n = A.shape[0]
    ld = ld or n
    buf = np.zeros((n, ld), np.complex128)
    buf[:, :n] = A
    d = torch.tensor(buf, dtype=torch.complex128, device="cuda")
    rc, health = B.bem_dense_invert(ctx, d.data_ptr(), n, ld)
    torch.cuda.synchronize()
    return rc, health, d.cpu().numpy()[:, :n]


def _well_posed(n, seed):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return A + (2.0 + 0.5j) * np.eye(n)


@pytest.mark.parametrize("n,ld", [(1, 1), (63, 63), (64, 70), (300, 300), (513, 520)])
def test_inverse_matches_lapack(torch_mod, ctx, n, ld):
    """Sizes below one panel, one panel, a ragged group of four (300 = 4 x 64 + 44) and more than
    one group (513 rows: two groups, the last panel of one row), with padded leading dimensions."""
    A = _well_posed(n, 7 + n)
    rc, (ratio, probe), Ainv = _invert(torch_mod, ctx, A, ld)
    assert rc == B.BEM_OK
    ref = np.linalg.inv(A)
    err = np.linalg.norm(Ainv - ref) / np.linalg.norm(ref)
    print(f"n {n}: rel err vs LAPACK {err:.2e}, pivot ratio {ratio:.2e}, probe {probe:.2e}")
    assert err < 1e-13
    assert 1e-3 < ratio <= 1.0 + 1e-12 or n == 1
    assert probe < 1e-13


def test_zero_leading_pivot_fails(torch_mod, ctx):
    """Rows 0 and 1 of a well-posed matrix swapped, its (0,0) entry zero: non-singular, but its
    first pivot is 0, so the elimination without pivoting must refuse it."""
    A = _well_posed(200, 3)
    A[0, 0] = 0.0
    A[[0, 1]] = A[[1, 0]]
    A[0, 0] = 0.0
    assert np.linalg.cond(A) < 1e4
    rc, (ratio, probe), _ = _invert(torch_mod, ctx, A)
    print(f"pivot ratio {ratio}, probe {probe}")
    assert rc == B.BEM_E_NUMERIC
    assert not (ratio >= 1e-12)


def test_tiny_leading_pivot_fails(torch_mod, ctx):
    """A leading 2 x 2 block [[1e-15, 1], [1, 1]] (well conditioned, but its first pivot is 1e-15 of
    the block): growth of 1e15 without pivoting; the pivot watch and the probe both see it."""
    A = _well_posed(150, 5) * 1e-3
    A[:2, :2] = [[1e-15, 1.0], [1.0, 1.0]]
    rc, (ratio, probe), _ = _invert(torch_mod, ctx, A)
    print(f"pivot ratio {ratio:.2e}, probe {probe:.2e}")
    assert rc == B.BEM_E_NUMERIC
    assert ratio < 1e-12


def test_singular_matrix_fails(torch_mod, ctx):
    """Rank 99 of 100 (the last column a combination of the others)."""
    A = _well_posed(100, 11)
    A[:, -1] = A[:, :-1] @ np.linspace(0.1, 1.0, 99)
    rc, (ratio, probe), _ = _invert(torch_mod, ctx, A)
    print(f"pivot ratio {ratio:.2e}, probe {probe:.2e}")
    assert rc == B.BEM_E_NUMERIC


def test_nonfinite_entry_fails(torch_mod, ctx):
    A = _well_posed(96, 13)
    A[70, 20] = np.nan
    rc, (ratio, probe), _ = _invert(torch_mod, ctx, A)
    assert rc == B.BEM_E_NUMERIC
    assert np.isnan(probe) or np.isnan(ratio)


def test_invalid_arguments(torch_mod, ctx):
    d = torch_mod.zeros((4, 4), dtype=torch_mod.complex128, device="cuda")
    with pytest.raises(B.BemError):
        B.bem_dense_invert(ctx, d.data_ptr(), 4, 3)
    with pytest.raises(B.BemError):
        B.bem_dense_invert(ctx, 0, 4, 4)
