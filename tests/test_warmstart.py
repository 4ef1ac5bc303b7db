"""Host-side pieces of the warm start from a smaller problem: the leading
principal submatrix of an upper-triangle CSR equals the dense principal block,
and the padded start block keeps the small solution above zeros."""
import numpy as np
import pytest

import synthgen as sg
from oracle import sparse as osp

ws = pytest.importorskip("paper_2305_15552_amd.warmstart")


@pytest.mark.parametrize("n_sub", [1, 37, 500, 1000])
def test_principal_csr_is_the_dense_block(n_sub):
    spec = sg.MatrixSpec(1000, 5, 8, 0.3, 3)
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSym(spec.n, rp, ci, v).dense()
    a, b, c = ws.principal_csr(rp, ci, v, n_sub)
    assert a.dtype == np.int64 and b.dtype == np.int32 and c.dtype == np.float32
    assert np.array_equal(osp.HalfSym(n_sub, a, b, c).dense(), H[:n_sub, :n_sub])


def test_principal_csr_with_empty_rows_and_padding():
    rp = np.array([0, 1, 1, 3], dtype=np.int64)
    ci = np.array([0, 1, 2], dtype=np.int32)
    v = np.array([1.0, 2.0, 3.0], dtype=np.float32)
    a, b, c = ws.principal_csr(rp, ci, v, 2)
    assert list(a) == [0, 1, 1] and list(b) == [0] and list(c) == [1.0]
    Xs = np.arange(6, dtype=np.float32).reshape(3, 2)
    X = ws.padded_start(Xs, 5)
    assert X.shape == (5, 2) and np.array_equal(X[:3], Xs) and not X[3:].any()
