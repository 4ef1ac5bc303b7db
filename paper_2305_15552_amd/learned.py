"""Training data and training for the learned preconditioner, driven through the
C-ABI only (every step runs in libhyeig's kernels; torch holds device memory).

Samples come from the solver itself: LOBPCG with the shifted-diagonal
preconditioner is run for a few iteration counts from the same start block,
and for each resulting Ritz block ``hyeig_mlp_labels`` computes the residual
features and the correction-equation targets (MINRES on the GPU).
"""
from __future__ import annotations

import numpy as np

from . import hyeig as hy


def hnorm_estimate(ctx, M, X0):
    """||H||_2 estimate of the library (30-step Lanczos), from a zero-iteration solve."""
    p = hy.params_default(k=1, nb=1, method=hy.LOBPCG, tol=1.0, hnorm=0.0, maxiter=0)
    _, _, rep, _, _ = hy.solve_lowest_k(ctx, M, p, X0[:, :1].clone())
    return rep.hnorm_used


def collect_samples(ctx, mats, nb=8, k=8, snapshots=(2, 4, 8, 16, 32), steps=20):
    """mats: iterable of (Matrix with row statistics, X0 FP32 n x nb device tensor).
    One sample per (row, column) of the k leading columns at each snapshot (the
    LOBPCG state after that many iterations): 5 snapshots of 8 columns of an
    n = 8192 matrix give about 3.3e5 samples per matrix.  (Nineteen snapshots,
    2, 4, ..., 38, give the ~1e7 samples of eight matrices; the network trained
    on them preconditioned worse.)
    Returns (features [N x 4], targets [N]) as FP32 device tensors."""
    import torch
    feats, targs = [], []
    for M, X0 in mats:
        hn = hnorm_estimate(ctx, M, X0)
        for it in snapshots:
            p = hy.params_default(k=k, nb=nb, method=hy.LOBPCG, tol=1e-6, hnorm=hn, maxiter=it,
                                  precision=hy.PREC_F32, precond=hy.PRECOND_JACOBI)
            X = X0.clone()
            hy.solve_lowest_k(ctx, M, p, X)
            F, T, _ = hy.mlp_labels(ctx, M, X[:, :k].contiguous(), hn, steps)
            ok = torch.isfinite(T) & torch.isfinite(F).all(dim=1)
            feats.append(F[ok])
            targs.append(T[ok])
    return torch.cat(feats).contiguous(), torch.cat(targs).contiguous()


def train(ctx, F, T, epochs=20, batch=65536, lr=1e-3, seed=0, init_seed=0, clip=None):
    """A fresh MLP trained by the library's Adam on (F, T); targets optionally
    clipped to [-clip, clip].  Returns (Mlp, per-epoch losses)."""
    import torch
    if clip is not None:
        T = torch.clamp(T, -clip, clip).contiguous()
    rng = np.random.default_rng(init_seed)
    p = np.zeros(hy.MLP_NPARAM)
    p[:256] = rng.uniform(-1, 1, 256) * np.sqrt(6.0 / 4)
    p[320:384] = rng.uniform(-1, 1, 64) * np.sqrt(6.0 / 64)
    mlp = hy.Mlp(ctx, p)
    losses = mlp.train(F, T, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return mlp, losses
