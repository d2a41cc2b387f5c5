"""Seeded generators: closed-form sizes, determinism, recipe properties."""
import numpy as np
import pytest

from paper_2509_07690_amd import synth


@pytest.mark.parametrize("dim,points,side", [(2, 5, 64), (2, 9, 33), (3, 7, 12), (3, 27, 9)])
def test_grid_nnz_closed_form(dim, points, side):
    pat = synth.grid2d(side, points) if dim == 2 else synth.grid3d(side, points)
    assert pat.n == side ** dim
    assert pat.nnz == synth.grid_nnz_closed_form(dim, points, side)
    # sorted, unique, diagonal present, symmetric pattern
    for i in range(0, pat.n, max(1, pat.n // 50)):
        c = pat.col[pat.row_ptr[i]:pat.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    d = pat.to_dense() if pat.n <= 1200 else None
    if d is not None:
        mask = np.zeros((pat.n, pat.n), bool)
        mask[pat.rows(), pat.col] = True
        assert np.array_equal(mask, mask.T)


def test_config0_values_and_rhs():
    w = synth.config(0)
    A = w.A
    assert A.n == 4096 and A.nnz == 20224
    dpos = A.diag_positions()
    d = A.val[dpos]
    assert np.all((d >= 4.0) & (d <= 5.0))
    off = np.delete(A.val, dpos)
    assert np.all((off >= -1.3) & (off <= -0.7))
    assert np.allclose(A.matvec(w.x_true), w.b)
    w2 = synth.config(0)
    assert np.array_equal(w.A.val, w2.A.val) and np.array_equal(w.b, w2.b)


def test_circuit_powerlaw_recipe():
    pat = synth.circuit_powerlaw_pattern(200000, 100)
    assert abs(pat.nnz / pat.n - 5.0) < 0.01
    assert np.all(pat.diag_positions() >= 0)
    deg = np.bincount(pat.col, minlength=pat.n)
    assert deg.max() <= 2001
    A = synth.dominant_values(pat, 1100)
    dpos = A.diag_positions()
    off = np.abs(A.val.copy())
    off[dpos] = 0
    s = np.bincount(A.rows(), weights=off, minlength=A.n)
    assert np.allclose(A.val[dpos], np.where(s > 0, 1.5 * s, 1.5))


def test_batch_member_shapes():
    for m in (0, 1, 2, 3):
        w = synth.batch_member(m)
        if m % 2 == 0:
            assert 2000 <= w.A.n <= 50000
            per_row = np.diff(w.A.row_ptr)
            assert per_row.max() <= 8 and per_row.min() >= 1
        else:
            s = int(round(np.sqrt(w.A.n)))
            assert s * s == w.A.n and 32 <= s <= 160
            assert w.A.nnz == synth.grid_nnz_closed_form(2, 9, s)
        A0 = w.extra["analyze_values"]
        assert np.array_equal(A0.col, w.A.col) and not np.array_equal(A0.val, w.A.val)
