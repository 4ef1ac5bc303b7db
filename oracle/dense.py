"""Small FP64 problems of the hybrid eigensolver.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotSPD(Exception):
    """Cholesky factorisation of a Gram matrix failed."""


def cholesky_upper(G):
    """R upper triangular with R^T R = G (raises NotSPD)."""
    G = 0.5 * (G + G.T)
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError as e:
        raise NotSPD(str(e))
    return L.T


def cholqr(X, passes=1):
    """CholeskyQR (Alg. 3, on the start block and on each filtered block): G = X^T X, G = R^T R, Q = X R^{-1}.
    With passes=2 the factorisation is repeated on Q (CholQR2) and R is the
    product of both factors.  Returns (Q, R)."""
    Q = np.asarray(X, dtype=np.float64)
    Rtot = np.eye(Q.shape[1])
    for _ in range(passes):
        R = cholesky_upper(Q.T @ Q)
        Q = sla.solve_triangular(R, Q.T, trans="T", lower=False).T
        Rtot = R @ Rtot
    return Q, Rtot


def rayleigh_ritz(A, B=None, nwant=None):
    """Rayleigh-Ritz on the projected pencil (A, B): the nwant leftmost
    eigenpairs of A c = theta B c with C^T B C = I (eq. (rreig); eq. (trideig)
    and (btrideig) when B = I).  Returns (theta ascending, C)."""
    A = 0.5 * (A + A.T)
    k = A.shape[0]
    nwant = k if nwant is None else nwant
    if B is None:
        w, V = sla.eigh(A, subset_by_index=[0, nwant - 1])
    else:
        B = 0.5 * (B + B.T)
        w, V = sla.eigh(A, B, subset_by_index=[0, nwant - 1])
    return w, V


def diis_coefficients(Bmat):
    """DIIS residual minimisation (eq. (xsum)-(rmm)): minimise
    || sum_l alpha_l r^(l) ||^2 subject to sum_l alpha_l = 1, given the Gram
    matrix Bmat[a, b] = <r^(a), r^(b)> of the window.  Solved as the bordered
    system [B 1; 1^T 0][alpha; mu] = [0; 1] after scaling B by its largest
    diagonal entry; least squares (rcond 1e-14) when that system is singular.
    The paper's substitution form (alpha_last = 1 - sum of the others) gives
    the same minimiser."""
    B = np.asarray(Bmat, dtype=np.float64)
    s = B.shape[0]
    if s == 1:
        return np.ones(1)
    B = 0.5 * (B + B.T)
    scale = np.max(np.abs(np.diag(B)))
    if scale > 0:
        B = B / scale
    M = np.zeros((s + 1, s + 1))
    M[:s, :s] = B
    M[:s, s] = 1.0
    M[s, :s] = 1.0
    rhs = np.zeros(s + 1)
    rhs[s] = 1.0
    try:
        sol = np.linalg.solve(M, rhs)
        if not np.all(np.isfinite(sol)):
            raise np.linalg.LinAlgError
    except np.linalg.LinAlgError:
        sol = np.linalg.lstsq(M, rhs, rcond=1e-14)[0]
    return sol[:s]


def rr_2x2(A, B):
    """The 2x2 Rayleigh-Ritz of RMM-DIIS (eq. (rr), (xuwg)): the eigenvector g
    of the smaller eigenvalue of the pencil (A, B), scaled so g^T B g = 1 and
    oriented so that (B g)_0 > 0.  Returns (theta, g)."""
    w, V = rayleigh_ritz(A, B, nwant=1)
    Bs = 0.5 * (B + B.T)
    g = V[:, 0]
    g = g / np.sqrt(g @ Bs @ g)
    # the sign of g is free; the DIIS combination of eq. (xsum) needs the
    # iterates oriented alike, so the new vector keeps a positive overlap with
    # the first basis vector (x~): (B g)_0 > 0
    if (Bs @ g)[0] < 0:
        g = -g
    return float(w[0]), g


def switch_tau(theta_now, theta_prev):
    """Switch metric of eq. (switchtau): the 1/n_ev factor sits outside the
    square root, as printed."""
    a = np.asarray(theta_now, dtype=np.float64)
    b = np.asarray(theta_prev, dtype=np.float64)
    return float(np.sqrt(np.sum(((a - b) / a) ** 2)) / a.size)


def effective_spmv(spmv_count, spmm_gflops, spmv_gflops):
    """Effective SpMV count (Section 4.2): SpMV count divided by the ratio of
    SpMM to SpMV throughput."""
    return spmv_count / (spmm_gflops / spmv_gflops)
