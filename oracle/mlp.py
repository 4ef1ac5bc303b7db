"""Learned per-row preconditioner: an MLP 4 -> 64 -> 1 (ReLU) applied entry by
entry to a residual block, trained to reproduce approximate solutions of the
correction equation (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper leaves the preconditioner K of LOBPCG open (Section 2.3, the
preconditioned residual block of eq. (wblock)); this learned K is a project
addition, not the paper's method.  Every definition below is a reading:

  parameters (385, FP32 master copy): W1[64][4], b1[64], w2[64], b2
      out(f) = w2 . relu(W1 f + b1) + b2

  features of entry (k, j) of a residual block R (column j has Ritz value
  theta_j), sample index k * ncol + j:
      f0 = (d_k - theta_j) / ||H||_2
      f1 = r_kj / ||r_j||_2 * sqrt(n)
      f2 = sum_l |H_kl| / ||H||_2
      f3 = nnz(row k of H) / mean over rows of nnz(row k of H)

  target: t_j = MINRES_20( P (H - theta_j I) P, -P r_j ),  P = I - X X^T,
      tau_kj = t_kj ||H||_2 sqrt(n) / ||r_j||_2
  (dimensionless: the shifted-diagonal preconditioner corresponds to
  tau = f1 / f0)

  apply: w_kj = out(f_kj) ||r_j||_2 / (||H||_2 sqrt(n))
"""
from __future__ import annotations

import numpy as np

NH = 64
NF = 4
NPARAM = NH * NF + 2 * NH + 1


def unpack(p):
    """(W1 [64 x 4], b1 [64], w2 [64], b2) views of the flat parameter vector."""
    p = np.asarray(p, dtype=np.float64)
    return p[:NH * NF].reshape(NH, NF), p[NH * NF:NH * NF + NH], p[NH * NF + NH:NH * NF + 2 * NH], p[-1]


def init_params(seed=0):
    """He-style initial weights (uniform, fan-in scaled), zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    p[:NH * NF] = rng.uniform(-1, 1, NH * NF) * np.sqrt(6.0 / NF)
    p[NH * NF + NH:NH * NF + 2 * NH] = rng.uniform(-1, 1, NH) * np.sqrt(6.0 / NH)
    return p


def forward(p, F):
    """out_i = w2 . relu(W1 f_i + b1) + b2 for the rows f_i of F (N x 4)."""
    W1, b1, w2, b2 = unpack(p)
    F = np.asarray(F, dtype=np.float64)
    h = np.maximum(F @ W1.T + b1, 0.0)
    return h @ w2 + b2


def loss_grad(p, F, t):
    """L = mean_i (out_i - t_i)^2 and dL/dp (385) by backpropagation."""
    W1, b1, w2, b2 = unpack(p)
    F = np.asarray(F, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    N = F.shape[0]
    pre = F @ W1.T + b1
    h = np.maximum(pre, 0.0)
    out = h @ w2 + b2
    e = out - t
    L = float(np.mean(e * e))
    go = 2.0 * e / N                      # dL/dout_i
    g_w2 = h.T @ go
    g_b2 = go.sum()
    gpre = np.outer(go, w2) * (pre > 0)   # dL/dpre_ih
    g_W1 = gpre.T @ F
    g_b1 = gpre.sum(axis=0)
    return L, np.concatenate([g_W1.ravel(), g_b1, g_w2, [g_b2]])


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, with bias correction); step counts from
    1.  Returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(d, theta, R, rowabs, rownnz, hnorm):
    """N x 4 features (N = n * ncol, sample k * ncol + j) of the residual block R."""
    R = np.asarray(R, dtype=np.float64)
    n, ncol = R.shape
    rn = np.linalg.norm(R, axis=0)
    rn = np.where(rn > 0, rn, 1.0)
    F = np.empty((n, ncol, NF))
    F[:, :, 0] = (np.asarray(d, dtype=np.float64)[:, None] - np.asarray(theta)[None, :]) / hnorm
    F[:, :, 1] = R / rn[None, :] * np.sqrt(n)
    F[:, :, 2] = (np.asarray(rowabs, dtype=np.float64) / hnorm)[:, None]
    nz = np.asarray(rownnz, dtype=np.float64)
    F[:, :, 3] = (nz / nz.mean())[:, None]
    return F.reshape(n * ncol, NF)


def minres(apply, b, steps, tol=0.0):
    """MINRES of Paige and Saunders (1975) for a symmetric, possibly indefinite
    operator: Lanczos tridiagonalisation with the least-squares problem solved
    by Givens rotations, so ||b - A x_k|| is minimised over the k-th Krylov
    space.  No preconditioner.  Returns (x, [|phibar_k|]) -- the recurrence's
    residual norms."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    beta1 = float(np.linalg.norm(b))
    if beta1 == 0.0:
        return x, [0.0]
    r1 = b.copy()
    r2 = b.copy()
    y = b.copy()
    oldb = 0.0
    beta = beta1
    dbar = 0.0
    epsln = 0.0
    phibar = beta1
    cs, sn = -1.0, 0.0
    w = np.zeros_like(b)
    w2 = np.zeros_like(b)
    hist = [beta1]
    for k in range(steps):
        v = y / beta
        y = apply(v)
        if k > 0:
            y = y - (beta / oldb) * r1
        alfa = float(v @ y)
        y = y - (alfa / beta) * r2
        r1, r2 = r2, y
        oldb = beta
        beta = float(np.linalg.norm(r2))
        oldeps = epsln
        delta = cs * dbar + sn * alfa
        gbar = sn * dbar - cs * alfa
        epsln = sn * beta
        dbar = -cs * beta
        gamma = max(np.hypot(gbar, beta), np.finfo(float).tiny)
        cs, sn = gbar / gamma, beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        hist.append(abs(phibar))
        if beta == 0.0 or abs(phibar) <= tol * beta1:
            break
    return x, hist


def correction_solutions(H, X, theta, R, steps=20):
    """t_j = MINRES_steps(P (H - theta_j I) P, -P r_j) with P = I - X X^T
    (X orthonormal, the current Ritz block), one column at a time."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    T = np.zeros_like(R)

    def proj(v):
        return v - X @ (X.T @ v)

    for j in range(R.shape[1]):
        th = float(theta[j])

        def apply(v, th=th):
            pv = proj(v)
            return proj(H @ pv - th * pv)

        T[:, j], _ = minres(apply, -proj(R[:, j]), steps)
    return T


def targets(T, R, hnorm):
    """tau_kj = t_kj ||H||_2 sqrt(n) / ||r_j||_2, flattened like ``features``."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    rn = np.linalg.norm(R, axis=0)
    rn = np.where(rn > 0, rn, 1.0)
    return (np.asarray(T) * hnorm * np.sqrt(n) / rn[None, :]).reshape(-1)


def precond_apply(p, R, theta, d, rowabs, rownnz, hnorm, net=None):
    """W = K^{-1} R with the learned K: w_kj = out(f_kj) ||r_j|| / (||H|| sqrt(n)).
    ``net`` (optional) replaces the network: a callable F (N x 4) -> out (N);
    with out = f1 / f0 the result is exactly the shifted diagonal r_kj / (d_k -
    theta_j), the identity the dimensionless features are built for."""
    R = np.asarray(R, dtype=np.float64)
    n, ncol = R.shape
    F = features(d, theta, R, rowabs, rownnz, hnorm)
    out = (forward(p, F) if net is None else np.asarray(net(F), dtype=np.float64)).reshape(n, ncol)
    rn = np.linalg.norm(R, axis=0)
    return out * rn[None, :] / (hnorm * np.sqrt(n))
