"""Half-stored symmetric products and the tall-skinny dense block kernels (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The matrix H is given by its upper triangle U including the diagonal, as the
paper's Hamiltonians are stored by half (Section 3.1, Tables 2 and 3 count the
non-zeros in half the symmetric matrix), so H = U + U^T - diag(U).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class HalfSym:
    """H = U + U^T - diag(U) from the upper-triangle CSR (values promoted
    exactly from FP32 to FP64)."""

    def __init__(self, n, rowptr, colidx, vals):
        self.n = int(n)
        self.U = sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(colidx, dtype=np.int64),
                                np.asarray(rowptr, dtype=np.int64)), shape=(self.n, self.n))
        self.d = self.U.diagonal().astype(np.float64)
        self.UT = self.U.T.tocsr()  # strictly a transposed view, materialised once
        self.spmm_calls = 0
        self.spmv_count = 0

    def matmul(self, X):
        """Y = H X (the product every method of Section 2 is built on; LOBPCG
        needs only H W per iteration, eq. (upd1)-(upd2))."""
        X = np.asarray(X, dtype=np.float64)
        Y = self.U @ X + self.UT @ X
        if X.ndim == 1:
            Y -= self.d * X
            self.spmv_count += 1
        else:
            Y -= self.d[:, None] * X
            self.spmv_count += X.shape[1]
        self.spmm_calls += 1
        return Y

    __matmul__ = matmul

    def dense(self):
        """The full symmetric matrix as a dense array (small n only)."""
        A = self.U.toarray()
        return A + A.T - np.diag(np.diag(A))

    def row_abs_sums(self):
        """Full-row 1-norms sum_j |H_kj| of the symmetric matrix."""
        a = abs(self.U)
        return np.asarray(a.sum(axis=1)).ravel() + np.asarray(a.sum(axis=0)).ravel() - np.abs(self.d)

    def row_nnz(self):
        """Stored entries of each full symmetric row."""
        s = (self.U != 0).astype(np.int64)
        return (np.asarray(s.sum(axis=1)).ravel() + np.asarray(s.sum(axis=0)).ravel()
                - (self.d != 0).astype(np.int64))


def spmm_sym(n, rowptr, colidx, vals, X):
    """Y = (U + U^T - diag U) X in FP64, straight from the definition."""
    return HalfSym(n, rowptr, colidx, vals).matmul(X)


def gram(A, B):
    """G = A^T B for tall-skinny blocks (the level-3 products that form the
    projected matrices S^T H S and S^T S, eq. (rreig), and the block
    Gram-Schmidt coefficients of eq. (bgs))."""
    return np.asarray(A, dtype=np.float64).T @ np.asarray(B, dtype=np.float64)


def block_update(S, C, beta=0.0, Y=None):
    """Y <- S C + beta Y (the block updates of eq. (xupd), (pupd), (upd1),
    (upd2) and the projection W - V G of eq. (bgs))."""
    out = np.asarray(S, dtype=np.float64) @ np.asarray(C, dtype=np.float64)
    if Y is not None and beta != 0.0:
        out = out + beta * np.asarray(Y, dtype=np.float64)
    return out


def residual(HX, X, theta):
    """R = H X - X Theta (Alg. 2) and the column 2-norms."""
    R = np.asarray(HX, dtype=np.float64) - np.asarray(X, dtype=np.float64) * np.asarray(theta)[None, :]
    return R, np.linalg.norm(R, axis=0)


def jacobi_apply(R, d, theta, floor):
    """Shifted diagonal preconditioner W = K^{-1} R (eq. (wblock)), K_j =
    diag(d) - theta_j I with |d_k - theta_j| floored at ``floor``.  The paper
    asks only that K approximate H and names no particular one; this is the
    reading used."""
    den = np.maximum(np.abs(np.asarray(d)[:, None] - np.asarray(theta)[None, :]), floor)
    return np.asarray(R, dtype=np.float64) / den


def product_rows(n, row0, rowptr, colidx, vals, X, rows):
    """Rows ``rows`` of H X computed from a band of upper-triangle CSR rows
    only: the CSR holds rows row0, row0+1, ... (local rowptr), and must include
    every row k <= max(rows) whose entries can reach a requested column (for the
    banded matrices: the band before the first requested row).  The same sum as
    ``HalfSym.matmul`` restricted to the requested rows:
        y_i = sum_{j >= i} u_ij x_j + sum_{k < i} u_ki x_k."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    nloc = rowptr.size - 1
    U = sp.csr_matrix((vals, colidx, rowptr), shape=(nloc, n))
    want = np.zeros(n, dtype=bool)
    want[rows] = True
    Y = np.zeros((rows.size, X.shape[1]))
    pos = {int(r): q for q, r in enumerate(rows)}
    # direct part: rows of U that are requested
    for r in rows:
        lr = int(r) - row0
        a, b = rowptr[lr], rowptr[lr + 1]
        Y[pos[int(r)]] += vals[a:b] @ X[colidx[a:b]]
    # transposed part: entries (k, i) with i requested and k < i
    coo = U.tocoo()
    k = coo.row + row0
    i = coo.col
    sel = want[i] & (k < i)
    for kk, ii, vv in zip(k[sel], i[sel], coo.data[sel]):
        Y[pos[int(ii)]] += vv * X[kk]
    return Y



# ---------------------------------------------------------------------------
# the same product on all host threads (plain C with OpenMP, halfsym_omp.c)
# ---------------------------------------------------------------------------
_HERE = __import__("os").path.dirname(__import__("os").path.abspath(__file__))
_LIB = None


def build_native(force=False):
    """Compiles halfsym_omp.c into oracle/libhalfsym_omp.so with gcc -fopenmp."""
    import os
    import subprocess
    src = os.path.join(_HERE, "halfsym_omp.c")
    out = os.path.join(_HERE, "libhalfsym_omp.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", src, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("oracle build failed: %s\n%s" % (" ".join(cmd), r.stdout + r.stderr))
        os.replace(tmp, out)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        import ctypes as C
        lib = C.CDLL(build_native())
        p = C.c_void_p
        lib.half_lower.restype = C.c_int64
        lib.half_lower.argtypes = [C.c_int64, p, p, p, p, p, p]
        lib.half_matmul.restype = None
        lib.half_matmul.argtypes = [C.c_int64, p, p, p, p, p, p, C.c_int, p, C.c_int64, p, C.c_int64, C.c_int]
        lib.half_threads.restype = C.c_int
        _LIB = lib
    return _LIB


class HalfSymOMP:
    """H = U + U^T - diag(U) applied by the plain C loop of halfsym_omp.c on
    all host threads (FP32 values promoted exactly, FP64 sums):
        y_i = sum_{j >= i} u_ij x_j + sum_{k < i} u_ki x_k,
    the second sum from the strictly lower triangle stored once as CSR.  The
    same sums as ``HalfSym.matmul`` (pinned against it in the tests); meant for
    the large matrices, where scipy's single-threaded products are too slow.
    ``threads`` <= 0: OpenMP's default."""

    def __init__(self, n, rowptr, colidx, vals, threads=0):
        self.n = int(n)
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        self.vals = np.ascontiguousarray(vals, dtype=np.float32)
        nnz = int(self.rowptr[-1])
        self.lrowptr = np.empty(self.n + 1, dtype=np.int64)
        self.lcol = np.empty(nnz, dtype=np.int32)
        self.lval = np.empty(nnz, dtype=np.float32)
        lib = _lib()
        nl = lib.half_lower(self.n, self.rowptr.ctypes.data, self.colidx.ctypes.data, self.vals.ctypes.data,
                            self.lrowptr.ctypes.data, self.lcol.ctypes.data, self.lval.ctypes.data)
        if nl < 0:
            raise MemoryError("half_lower")
        self.lcol = self.lcol[:nl]
        self.lval = self.lval[:nl]
        self.threads = int(threads)
        self.d = np.zeros(self.n)
        r = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        on = self.colidx == r
        self.d[r[on]] = self.vals[on]
        self.spmm_calls = 0
        self.spmv_count = 0

    def nthreads(self):
        return self.threads if self.threads > 0 else int(_lib().half_threads())

    def matmul(self, X):
        X = np.asarray(X, dtype=np.float64)
        vec = X.ndim == 1
        X2 = np.ascontiguousarray(X.reshape(self.n, -1))
        m = X2.shape[1]
        Y = np.empty((self.n, m))
        _lib().half_matmul(self.n, self.rowptr.ctypes.data, self.colidx.ctypes.data, self.vals.ctypes.data,
                           self.lrowptr.ctypes.data, self.lcol.ctypes.data, self.lval.ctypes.data, m,
                           X2.ctypes.data, m, Y.ctypes.data, m, self.threads)
        self.spmm_calls += 1
        self.spmv_count += m
        return Y.ravel() if vec else Y

    __matmul__ = matmul
