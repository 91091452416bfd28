"""The seeded input recipes: shapes, sizes, structure and reproducibility."""
import numpy as np
import pytest
import scipy.sparse as sp

import problems


def test_anisotropic_csr_full_size_structure():
    p = problems.anisotropic_csr(1024, seed=0)
    op = p.op
    assert op.n == 1_048_576
    assert op.nnz == 5_238_784
    assert op.row_ptr.dtype == np.int64 and op.col.dtype == np.int32
    # binary32-exact values
    assert np.array_equal(op.val, op.val.astype(np.float32).astype(np.float64))
    A = problems.to_scipy(op)
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - d
    assert np.all(d >= off)                       # weak diagonal dominance
    assert np.count_nonzero(d > off) >= 4 * 1024 - 4  # strict on the boundary rows


def test_anisotropic_csr_small_is_spd_and_symmetric():
    p = problems.anisotropic_csr(24, seed=3)
    A = problems.to_scipy(p.op)
    assert abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev[0] > 0
    np.testing.assert_allclose(A @ p.x_true, p.b, rtol=1e-14, atol=1e-14 * abs(p.b).max())


@pytest.mark.parametrize("n", [1000, 5000])
def test_banded_csr_structure(n):
    p = problems.banded_csr(n, seed=n)
    A = problems.to_scipy(p.op)
    assert abs(A - A.T).max() == 0.0
    rows = np.diff(p.op.row_ptr)
    assert rows.min() >= 2 and rows.mean() > 7
    i, j = A.nonzero()
    assert np.abs(i - j).max() <= 64
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - d
    assert np.all(d >= 1.01 * off * (1 - 1e-6))
    assert np.array_equal(p.op.val, p.op.val.astype(np.float32).astype(np.float64))


def test_batch_rectangles_recipe():
    batch = problems.batch_rectangles(512, seed=0)
    assert len(batch) == 512
    sides = np.array([(q.op.nx, q.op.ny) for q in batch])
    assert sides.min() >= 32 and sides.max() <= 256
    shifts = np.array([q.op.shift for q in batch])
    assert shifts.min() >= 0 and shifts.max() < 0.1
    for q in batch[:5]:
        assert q.sigma == pytest.approx(4.0 + q.op.shift)
        assert np.all(np.abs(q.b) <= 1)


def test_arrival_stream_recipe():
    s = problems.arrival_stream(40, rate_hz=10.0, seed=1, log10_max=4.5)
    t = np.array([a for a, _ in s])
    assert np.all(np.diff(t) > 0)
    kinds = {p.op.kind for _, p in s}
    assert kinds == {"3d7", "csr"}
    for _, p in s:
        assert 10 ** 2.9 <= p.op.n <= 10 ** 4.6
        assert p.jacobi and p.rtol == 1e-8


def test_seeded_reproducible():
    a = problems.poisson3d(10, seed=3)
    b = problems.poisson3d(10, seed=3)
    c = problems.poisson3d(10, seed=4)
    assert np.array_equal(a.b, b.b) and not np.array_equal(a.b, c.b)


def test_stencil_rhs_equals_kronecker_matvec():
    p = problems.poisson3d(9, seed=1)
    A = problems.to_scipy(p.op)
    np.testing.assert_allclose(A @ p.x_true, p.b, rtol=1e-14, atol=1e-14)
    q = problems.batch_rectangles(3, seed=2, side_min=5, side_max=9)[0]
    assert isinstance(problems.to_scipy(q.op), sp.csr_matrix)


def test_box_grid_rhs_equals_padded_stencil():
    # a non-cubic box (the shape of one slab of a split grid): b = A x_true
    # with A the 7-point stencil applied by explicit zero padding
    p = problems.poisson3d(8, ny=6, nz=4, seed=2)
    assert (p.op.nx, p.op.ny, p.op.nz, p.op.n) == (8, 6, 4, 192)
    x = np.pad(p.x_true.reshape(4, 6, 8), 1)
    ax = 6.0 * x[1:-1, 1:-1, 1:-1] - (x[:-2, 1:-1, 1:-1] + x[2:, 1:-1, 1:-1] + x[1:-1, :-2, 1:-1] +
                                      x[1:-1, 2:, 1:-1] + x[1:-1, 1:-1, :-2] + x[1:-1, 1:-1, 2:])
    np.testing.assert_allclose(ax.ravel(), p.b, rtol=0, atol=1e-14)
