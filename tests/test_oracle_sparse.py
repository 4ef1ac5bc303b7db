"""Pins for oracle.sparse: brute force from the CSR entries, closed forms,
self-adjointness, explicit loops for the block kernels."""
import numpy as np
import pytest

import synthgen as sg
from oracle import sparse as osp


def _brute_dense(n, rp, ci, v):
    A = np.zeros((n, n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            j = ci[p]
            A[i, j] = float(v[p])
            A[j, i] = float(v[p])
    return A


@pytest.mark.parametrize("n", [64, 97, 300])
def test_spmm_sym_against_brute_force(n):
    spec = sg.MatrixSpec(n, 3, 4, 0.3, n)
    rp, ci, v = sg.gen_csr(spec)
    A = _brute_dense(n, rp, ci, v)
    X = sg.normal_block(n, 5, 9)
    Y = osp.spmm_sym(n, rp, ci, v, X)
    # plain triple loop for a few rows
    for i in [0, n // 2, n - 1]:
        for c in range(5):
            s = sum(A[i, j] * X[j, c] for j in range(n))
            assert abs(Y[i, c] - s) < 1e-12 * (1 + np.abs(A[i]).sum())
    np.testing.assert_allclose(Y, A @ X, rtol=0, atol=1e-12)
    H = osp.HalfSym(n, rp, ci, v)
    np.testing.assert_allclose(H.dense(), A, rtol=0, atol=0)
    np.testing.assert_allclose(H.row_abs_sums(), np.abs(A).sum(axis=1), rtol=1e-14)
    np.testing.assert_array_equal(H.row_nnz(), (A != 0).sum(axis=1))


def test_spmm_sym_closed_forms():
    n = 50
    # diagonal only: H X = d * X
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    d = np.linspace(-3, 4, n).astype(np.float32)
    X = sg.normal_block(n, 3, 1)
    np.testing.assert_allclose(osp.spmm_sym(n, rp, ci, d, X), d.astype(np.float64)[:, None] * X, atol=1e-15)
    # tridiagonal Toeplitz a on the diagonal, b off it: (HX)_i = a x_i + b (x_{i-1} + x_{i+1})
    a, b = 2.0, -1.0
    rp = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        cols.append(i); vals.append(a)
        if i + 1 < n:
            cols.append(i + 1); vals.append(b)
        rp[i + 1] = len(cols)
    Y = osp.spmm_sym(n, rp, np.array(cols, np.int32), np.array(vals, np.float32), X)
    Xp = np.vstack([np.zeros((1, 3)), X, np.zeros((1, 3))])
    np.testing.assert_allclose(Y, a * X + b * (Xp[:-2] + Xp[2:]), atol=1e-14)


def test_spmm_sym_self_adjoint():
    spec = sg.MatrixSpec(1000, 5, 8, 0.3, 3)
    H = osp.HalfSym(spec.n, *sg.gen_csr(spec))
    X = sg.normal_block(spec.n, 4, 1)
    Z = sg.normal_block(spec.n, 4, 2)
    lhs = np.sum(X * (H @ Z))
    rhs = np.sum((H @ X) * Z)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_block_kernels_explicit_loops():
    A = sg.normal_block(40, 3, 1)
    B = sg.normal_block(40, 4, 2)
    G = osp.gram(A, B)
    for a in range(3):
        for b in range(4):
            assert abs(G[a, b] - sum(A[r, a] * B[r, b] for r in range(40))) < 1e-12
    C = sg.normal_block(3, 4, 3)
    Y0 = sg.normal_block(40, 4, 4)
    Y = osp.block_update(A, C, 0.5, Y0)
    for r in [0, 17, 39]:
        for c in range(4):
            assert abs(Y[r, c] - (sum(A[r, q] * C[q, c] for q in range(3)) + 0.5 * Y0[r, c])) < 1e-12
    R, nr = osp.residual(B, B * 2.0, np.array([0.5, 0.5, 0.5, 0.5]))
    np.testing.assert_allclose(R, 0.0, atol=0)
    d = np.linspace(0, 1, 40)
    th = np.array([0.5, 0.1, 2.0, 0.49])
    W = osp.jacobi_apply(B, d, th, 0.05)
    for r in [0, 19, 20, 39]:
        for c in range(4):
            assert W[r, c] == B[r, c] / max(abs(d[r] - th[c]), 0.05)


def test_product_rows_from_a_band_equal_full_rows():
    # rows of H X from only the CSR band that reaches them equal the full product's rows
    spec = sg.MatrixSpec(2048, 6, 8, 0.3, 52)
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSym(spec.n, rp, ci, v)
    X = sg.normal_block(spec.n, 3, 53)
    full = H @ X
    J = 40  # block row; the band of 8 block rows before it reaches its columns
    i0 = J - spec.w
    brp, bci, bv = sg.gen_block_rows(spec, i0, J + 1)
    rows = np.arange(32 * J, 32 * J + 32)
    Y = osp.product_rows(spec.n, 32 * i0, brp, bci, bv, X, rows)
    np.testing.assert_allclose(Y, full[rows], rtol=1e-13, atol=1e-13 * np.abs(full).max())


@pytest.mark.parametrize("n,m", [(97, 1), (300, 5), (4113, 16)])
def test_threaded_product_against_brute_force(n, m):
    """The oracle's C/OpenMP product (rows summed from U and from its strictly
    lower transpose) against the dense matrix built entry by entry, and the
    strictly lower CSR it builds against the transposed entries of U."""
    spec = sg.MatrixSpec(n, 5, 20, 0.3, n + 7)
    rp, ci, v = sg.gen_csr(spec)
    Ht = osp.HalfSymOMP(n, rp, ci, v, threads=3)
    A = _brute_dense(n, rp, ci, v)
    X = sg.normal_block(n, m, 4)
    Y = Ht @ X
    ref = A @ X
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(A).sum(axis=1).max() * np.abs(X).max()
    y1 = Ht @ X[:, 0]
    assert y1.shape == (n,)
    assert np.abs(y1 - ref[:, 0]).max() <= 1e-13 * np.abs(A).sum(axis=1).max() * np.abs(X).max()
    # L holds exactly the strictly lower entries, rows ascending in column
    L = np.zeros((n, n))
    for i in range(n):
        cols = Ht.lcol[Ht.lrowptr[i]:Ht.lrowptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and np.all(cols < i)
        L[i, cols] = Ht.lval[Ht.lrowptr[i]:Ht.lrowptr[i + 1]]
    np.testing.assert_array_equal(L, np.tril(A, -1))
    np.testing.assert_array_equal(Ht.d, np.diag(A))
