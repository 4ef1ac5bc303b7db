"""Warm starts from a smaller problem, the analogue of the paper's N_max - 2
start vectors (Section 1 counts the reuse of earlier approximations among the
block methods' strengths, and Section 3 starts from them): the leading
principal submatrix of H is the Hamiltonian of a smaller model space; its
lowest eigenvectors, padded with zeros, start the solve of the full problem.

Host-side data preparation only (slicing a CSR and padding a block): every
step of the solves runs in the library.
"""
from __future__ import annotations

import numpy as np


def principal_csr(rowptr, colidx, vals, n_sub):
    """The leading n_sub x n_sub block of an upper-triangle CSR (rows < n_sub,
    columns < n_sub), as (rowptr int64[n_sub+1], colidx int32, vals float32)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx)
    end = int(rowptr[n_sub])
    keep = colidx[:end] < n_sub
    # kept entries before each row start: the new row pointer (empty rows allowed)
    ck = np.zeros(end + 1, dtype=np.int64)
    np.cumsum(keep, out=ck[1:])
    rp = ck[rowptr[:n_sub + 1]]
    return rp, np.ascontiguousarray(colidx[:end][keep], dtype=np.int32), np.ascontiguousarray(
        np.asarray(vals)[:end][keep], dtype=np.float32)


def padded_start(X_sub, n):
    """n x m start block: X_sub in the leading rows, zeros below."""
    X_sub = np.asarray(X_sub, dtype=np.float32)
    X = np.zeros((n, X_sub.shape[1]), dtype=np.float32)
    X[:X_sub.shape[0]] = X_sub
    return X
