"""Plain FP64 iterative eigensolvers: LOBPCG, block Lanczos, batched RMM-DIIS
and the hybrids of Section 2.7 / Section 4.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The operator ``H`` is anything with ``H @ X`` (``oracle.sparse.HalfSym`` or a
dense array).  All arithmetic is float64.  Convergence uses the relative
residual ||H x - theta x|| / scale, scale = ||H||_2 (``norm="hnorm"``) or
|theta| (``norm="theta"``, the paper's form in Section 3.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import dense
from .sparse import jacobi_apply


def _apply(H, X):
    return H @ X


def _scale(theta, hnorm, norm):
    if norm == "theta":
        return np.abs(theta)
    return np.full_like(np.asarray(theta, dtype=np.float64), hnorm)


@dataclass
class Result:
    theta: np.ndarray
    X: np.ndarray
    HX: np.ndarray
    resid: np.ndarray            # relative residual of the returned pairs
    iters: int
    spmm: int                    # number of products H @ block
    spmv: int                    # number of vectors multiplied by H
    converged: bool
    history: list = field(default_factory=list)   # per-iteration relative residuals
    theta_hist: list = field(default_factory=list)
    tau_hist: list = field(default_factory=list)
    cond_hist: list = field(default_factory=list)
    events: list = field(default_factory=list)


def lobpcg(H, X0, k, tol=1e-6, maxiter=500, hnorm=1.0, norm="hnorm", precond="jacobi", d=None,
           jacobi_floor=None, stop=None, lock=True, state=None):
    """LOBPCG (Alg. 2) with the H X / H P recurrences of eq. (upd1)-(upd2), so
    the only product per iteration is H W (Section 2.3).

    X0: n x n_b start block.  k = n_ev leading columns tested for convergence.
    precond: "jacobi" (shifted diagonal, see ``jacobi_apply``), "none", or a
    callable (R, theta) -> W.
    stop: optional callable(it, theta, rel_resid) -> bool used by the hybrid
    switch (tested after the convergence test).
    Stabilisation (the paper cites stabilised variants without giving one):
      - soft locking (lock=True): a column whose relative residual is below tol
        stops contributing W and P columns to the subspace (it stays in X and is
        still updated by the Rayleigh-Ritz step);
      - columns of W are scaled to unit norm, and for the Rayleigh-Ritz step
        every column of S = [X W P] is scaled to unit norm (the same subspace,
        so the same Ritz pairs);
      - if that scaled Gram matrix of S is not positive definite or its
        condition number exceeds 1e12, P is dropped for that iteration; if that
        still fails, W is orthogonalised against X and orthonormalised;
      - if every column is locked while the leading k are not converged, the
        unconverged and the leading k columns are made active again.
    state: the ``state`` of an earlier Result to continue that iteration where
    it stopped (X, HX, P, HP, Ritz values, locked columns and the iteration
    count; X0 is then ignored and maxiter counts from the first run's start).
    The returned Result carries ``state`` for the same purpose."""
    if jacobi_floor is None:
        jacobi_floor = 1e-2 * hnorm
    if state is None:
        n, nb = X0.shape
        # Alg. 2 set-up: Rayleigh-Ritz on the start block.
        X, _ = np.linalg.qr(np.asarray(X0, dtype=np.float64))
        HX = _apply(H, X)
        spmm, spmv = 1, nb
        theta, C = dense.rayleigh_ritz(X.T @ HX)
        X, HX = X @ C, HX @ C
        P = HP = None
        active = np.ones(nb, dtype=bool)
        it = 0
    else:
        X, HX, P, HP = state["X"], state["HX"], state["P"], state["HP"]
        theta, active, it = state["theta"], state["active"].copy(), state["it"]
        n, nb = X.shape
        spmm, spmv = 0, 0
    res = Result(theta, X, HX, None, 0, spmm, spmv, False)
    prev_theta = None
    while True:
        R = HX - X * theta[None, :]
        rel = np.linalg.norm(R, axis=0) / _scale(theta, hnorm, norm)
        res.history.append(rel[:k].copy())
        res.theta_hist.append(theta[:k].copy())
        if prev_theta is not None:
            res.tau_hist.append(dense.switch_tau(theta[:k], prev_theta[:k]))
        prev_theta = theta.copy()
        if np.all(rel[:k] <= tol):
            res.converged = True
            break
        if stop is not None and stop(it, theta, rel):
            break
        if it >= maxiter:
            break
        it += 1
        if lock:
            active &= rel > tol
            if not active.any():
                active = (rel > tol) | (np.arange(nb) < k)
        idx = np.flatnonzero(active)
        na = idx.size
        # Alg. 2: W = K^{-1} R on the active columns.
        Ra = R[:, idx]
        if precond == "jacobi":
            W = jacobi_apply(Ra, d, theta[idx], jacobi_floor)
        elif precond == "none" or precond is None:
            W = Ra.copy()
        else:
            W = precond(Ra, theta[idx])
        W /= np.maximum(np.linalg.norm(W, axis=0), 1e-300)[None, :]
        HW = _apply(H, W)
        spmm += 1
        spmv += na
        use_p = P is not None
        for attempt in range(3):
            if use_p:
                S = np.hstack([X, W, P[:, idx]])
                HS = np.hstack([HX, HW, HP[:, idx]])
            else:
                S = np.hstack([X, W])
                HS = np.hstack([HX, HW])
            GS = S.T @ S
            GH = S.T @ HS
            GS, GH = 0.5 * (GS + GS.T), 0.5 * (GH + GH.T)
            sc = 1.0 / np.sqrt(np.maximum(np.diag(GS), 1e-300))
            GS = GS * sc[:, None] * sc[None, :]
            GH = GH * sc[:, None] * sc[None, :]
            ev = np.linalg.eigvalsh(GS)
            cond = ev[-1] / ev[0] if ev[0] > 0 else np.inf
            ok = np.isfinite(cond) and cond <= 1e12
            if ok:
                try:
                    theta_new, Cfull = dense.rayleigh_ritz(GH, GS, nb)
                    Cfull = Cfull * sc[:, None]
                    break
                except (np.linalg.LinAlgError, sla.LinAlgError):
                    ok = False
            if use_p:
                use_p = False
                res.events.append((it, "drop_P"))
            else:
                W = W - X @ (X.T @ W)
                W, _ = dense.cholqr(W, passes=2)
                HW = _apply(H, W)
                spmm += 1
                spmv += na
                res.events.append((it, "orth_W"))
        res.cond_hist.append(float(cond))
        theta = theta_new
        X, HX = S @ Cfull, HS @ Cfull
        # eq. (pupd), (upd2): the new search direction and its image.
        P, HP = S[:, nb:] @ Cfull[nb:], HS[:, nb:] @ Cfull[nb:]
    rel_final = np.linalg.norm(HX - X * theta[None, :], axis=0) / _scale(theta, hnorm, norm)
    res.theta, res.X, res.HX, res.resid = theta, X, HX, rel_final
    res.iters, res.spmm, res.spmv = it, spmm, spmv
    res.state = {"X": X, "HX": HX, "P": P, "HP": HP, "theta": theta, "active": active, "it": it}
    return res


def block_lanczos(H, X0, k, tol=1e-6, maxiter=200, hnorm=1.0, norm="hnorm", stop=None, nret=None):
    """Block Lanczos (Alg. 1) with full block Gram-Schmidt (eq. (bgs)) done as
    two classical passes, QR of W by CholeskyQR2, and the block tridiagonal T
    assembled from the diagonal blocks A_i = V_i^T H V_i and the QR factors
    R_{i+1} (no extra products, eq. (blanfac)).  Convergence uses the Ritz
    residual ||R_{i+1} E_i^T q|| (the quantity eq. (ritzest2) bounds).
    Returns X = V Q(:, :k) and H X from the block Lanczos relation; with nret
    > k, X and H X hold the nret leftmost Ritz pairs (as many as the basis has)
    and ``theta`` all of their Ritz values."""
    n, nb = X0.shape
    V1, _ = np.linalg.qr(np.asarray(X0, dtype=np.float64))
    Vs = [V1]
    As, Rs = [], []          # Rs[i] couples block i and i+1
    U = _apply(H, V1)
    spmm, spmv = 1, nb
    res = Result(None, None, None, None, 0, 0, 0, False)
    prev_theta = None
    it = 0
    while True:
        it += 1
        Vi = Vs[-1]
        Ai = Vi.T @ U
        Ai = 0.5 * (Ai + Ai.T)
        As.append(Ai)
        W = U - Vi @ Ai
        if len(Vs) > 1:
            W = W - Vs[-2] @ Rs[-1].T
        Vall = np.hstack(Vs)
        for _ in range(2):
            W = W - Vall @ (Vall.T @ W)
        try:
            Vn, Rn = dense.cholqr(W, passes=2)
        except dense.NotSPD:
            Vn, Rn = np.linalg.qr(W)
            res.events.append((it, "qr_fallback"))
        Rs.append(Rn)
        m = nb * it
        T = np.zeros((m, m))
        for b in range(it):
            T[b * nb:(b + 1) * nb, b * nb:(b + 1) * nb] = As[b]
            if b + 1 < it:
                T[(b + 1) * nb:(b + 2) * nb, b * nb:(b + 1) * nb] = Rs[b]
                T[b * nb:(b + 1) * nb, (b + 1) * nb:(b + 2) * nb] = Rs[b].T
        theta, Q = sla.eigh(T)
        kk = min(k, m)
        est = np.linalg.norm(Rn @ Q[-nb:, :kk], axis=0)
        rel = est / _scale(theta[:kk], hnorm, norm)
        res.history.append(rel.copy())
        res.theta_hist.append(theta[:kk].copy())
        if prev_theta is not None and prev_theta.size == kk:
            res.tau_hist.append(dense.switch_tau(theta[:kk], prev_theta))
        prev_theta = theta[:kk].copy()
        done = kk == k and np.all(rel <= tol)
        stopped = (not done) and stop is not None and kk == k and stop(it, theta, rel)
        if done or stopped or it >= maxiter:
            Vall = np.hstack(Vs)
            ne = k if nret is None else max(k, min(nret, m))
            X = Vall @ Q[:, :ne]
            HX = X * theta[None, :ne] + Vn @ (Rn @ Q[-nb:, :ne])
            res.theta, res.X, res.HX = theta[:ne], X, HX
            res.resid = rel
            res.converged = bool(done)
            break
        Vs.append(Vn)
        U = _apply(H, Vn)
        spmm += 1
        spmv += nb
    res.iters, res.spmm, res.spmv = it, spmm, spmv
    return res


def rmm_diis(H, X, k=None, HX=None, s_max=10, tol=1e-6, maxiter=300, hnorm=1.0, norm="hnorm",
             precond=None, residual_form="text", guard=False):
    """RMM-DIIS (Alg. 4) refining the columns of X simultaneously, the n_ev
    products of each sweep batched into one H @ block (Section 4.2).  Converged
    columns stay in the product but are no longer updated (the coupled variant
    of Section 4.2).

    Per column j and sweep i:
      i > 1: alpha from the DIIS problem over the last min(i, s_max) entries
             (eq. (xsum)-(rmm)); x~ = sum alpha x^(l), normalised; H x~ by
             linearity from the stored H x^(l) = r^(l) + theta^(l) x^(l);
             theta~ the Rayleigh quotient and r~ = H x~ - theta~ x~ (the text
             after eq. (rmm));  residual_form="sum" uses r~ = sum alpha r^(l)
             instead (the form printed in Alg. 4, kept for comparison);
      optional r~ <- K^{-1} r~ (precond callable (R, theta) -> W);
      2x2 Rayleigh-Ritz on span{x~, r~} (eq. (rr), (xuwg)); new residual;
      converged when ||r|| / scale < tol.
    guard=True stops early (converged=False, event "stagnation") when an
    unconverged column's residual exceeds 10x its best value so far, its best
    has not improved for 2*s_max sweeps, or its best has not halved over the
    last s_max sweeps, one DIIS window (where RMM-DIIS works it gains orders of
    magnitude in that many): the 2x2 Rayleigh-Ritz keeps the smaller root, so once the error
    of a column is dominated by lower eigenvectors the iteration drifts towards
    them (the paper notes that RMM-DIIS may converge to pairs other than the
    wanted ones).  The paper has no such guard; it is this project's reading.
    Returns a Result whose history has one row of relative residuals per sweep."""
    X = np.array(X, dtype=np.float64, copy=True)
    n, kk = X.shape
    k = kk if k is None else k
    spmm = spmv = 0
    if HX is None:
        HX = _apply(H, X)
        spmm, spmv = 1, kk
    HX = np.array(HX, dtype=np.float64, copy=True)
    nrm = np.linalg.norm(X, axis=0)
    X /= nrm[None, :]
    HX /= nrm[None, :]
    theta = np.einsum("ij,ij->j", X, HX)
    R = HX - X * theta[None, :]
    hist = [[(X[:, j].copy(), R[:, j].copy(), theta[j])] for j in range(kk)]
    done = np.zeros(kk, dtype=bool)
    rel = np.linalg.norm(R, axis=0) / _scale(theta, hnorm, norm)
    done[:] = rel <= tol
    res = Result(theta.copy(), X, HX, rel, 0, 0, 0, False)
    res.history.append(rel[:k].copy())
    Xt = X.copy()
    HXt = HX.copy()
    Rt = R.copy()
    best = rel.copy()
    best_it = np.zeros(kk, dtype=int)
    best_log = []          # the best residuals after each sweep
    it = 0
    while not np.all(done[:k]) and it < maxiter:
        it += 1
        thetat = theta.copy()
        for j in range(kk):
            if done[j] or it == 1:
                continue
            win = hist[j][-s_max:]
            rr = np.array([h[1] for h in win]).T           # n x s
            B = rr.T @ rr
            alpha = dense.diis_coefficients(B)
            xs = np.array([h[0] for h in win]).T
            hx = rr + xs * np.array([h[2] for h in win])[None, :]
            xt = xs @ alpha
            hxt = hx @ alpha
            nx = np.linalg.norm(xt)
            xt, hxt = xt / nx, hxt / nx
            tt = xt @ hxt
            if residual_form == "sum":
                rt = (rr @ alpha) / nx
            else:
                rt = hxt - tt * xt
            Xt[:, j], HXt[:, j], Rt[:, j], thetat[j] = xt, hxt, rt, tt
        if it == 1:
            Xt, HXt, Rt = X.copy(), HX.copy(), R.copy()
        Zt = Rt.copy()
        if precond is not None:
            Zt = precond(Rt, thetat)
        HZ = _apply(H, Zt)
        spmm += 1
        spmv += kk
        for j in range(kk):
            if done[j]:
                continue
            x, z, hx, hz = Xt[:, j], Zt[:, j], HXt[:, j], HZ[:, j]
            A = np.array([[x @ hx, x @ hz], [x @ hz, z @ hz]])
            Bm = np.array([[x @ x, x @ z], [x @ z, z @ z]])
            th, g = dense.rr_2x2(A, Bm)
            xn = g[0] * x + g[1] * z
            hxn = g[0] * hx + g[1] * hz
            rn = hxn - th * xn
            X[:, j], HX[:, j], R[:, j], theta[j] = xn, hxn, rn, th
            hist[j].append((xn.copy(), rn.copy(), th))
            if len(hist[j]) > s_max:
                hist[j].pop(0)
        rel = np.linalg.norm(R, axis=0) / _scale(theta, hnorm, norm)
        done |= rel <= tol
        res.history.append(rel[:k].copy())
        res.theta_hist.append(theta[:k].copy())
        improved = rel < best
        best = np.where(improved, rel, best)
        best_it = np.where(improved, it, best_it)
        best_log.append(best.copy())
        if guard:
            bad = (~done[:k]) & ((rel[:k] > 10 * best[:k]) | (it - best_it[:k] > 2 * s_max))
            w = s_max
            if len(best_log) > w:
                bad |= (~done[:k]) & (best[:k] > 0.5 * best_log[-1 - w][:k])
            if np.any(bad):
                res.events.append((it, "stagnation"))
                break
    res.theta, res.X, res.HX, res.resid = theta.copy(), X, HX, rel
    res.iters, res.spmm, res.spmv = it, spmm, spmv
    res.converged = bool(np.all(done[:k]))
    return res


def cheb_filter(H, X, HX, degree, c, e):
    """The Chebyshev filter of Section 2.4 applied to the columns of X:
    T_d((H - cI)/e) X with the first-kind polynomials of eq. (chebypoly)
    (T_0 = 1, T_1 = t, T_m = 2t T_{m-1} - T_{m-2}), by the three-term
    recurrence (Alg. 3, the inner loop).  HX = H X is given, so the filter
    costs degree - 1 products.  Returns (T_d((H - cI)/e) X, products)."""
    Q = np.asarray(X, dtype=np.float64)
    W = (np.asarray(HX, dtype=np.float64) - c * Q) / e      # T_1
    products = 0
    for _ in range(2, degree + 1):
        HW = _apply(H, W)
        products += 1
        Y = 2.0 * (HW - c * W) / e - Q                        # T_j = 2t T_{j-1} - T_{j-2}
        Q, W = W, Y
    return W, products


def spectrum_upper_bound(H, n, steps=10, start=None):
    """lambda_ub of Section 3 (the ChebFSI set-up): `steps` single-vector Lanczos
    steps (full re-orthogonalisation) from `start` (ones if None), then the
    largest Ritz pair (theta, u) of the tridiagonal matrix and
    lambda_ub = theta + ||H u - theta u||, the residual norm taken from the
    Lanczos relation (beta_m |last component of the Ritz vector|).
    Returns (lambda_ub, theta, residual norm, u, products)."""
    v = np.ones(n) if start is None else np.asarray(start, dtype=np.float64).copy()
    v = v / np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    for j in range(steps):
        w = _apply(H, V[-1])
        a = float(V[-1] @ w)
        w = w - a * V[-1] - (betas[-1] * V[-2] if betas else 0.0)
        Vm = np.array(V).T
        for _ in range(2):
            w = w - Vm @ (Vm.T @ w)
        b = float(np.linalg.norm(w))
        alphas.append(a)
        betas.append(b)
        if b == 0.0 or j == steps - 1:
            break
        V.append(w / b)
    m = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:m - 1], 1) + np.diag(betas[:m - 1], -1)
    th, S = np.linalg.eigh(T)
    rnorm = betas[m - 1] * abs(S[-1, -1])
    u = np.array(V[:m]).T @ S[:, -1]
    return float(th[-1] + rnorm), float(th[-1]), float(rnorm), u, m


def chebfsi(H, X0, k, degree=10, tol=1e-6, maxiter=200, hnorm=1.0, norm="hnorm", lam_ub=None, lam_f=None,
            lock=True, stop=None):
    """Chebyshev-filtered subspace iteration (Alg. 3).

    X0: n x n_b start block; k = n_ev leading pairs tested for convergence.
    lam_ub: upper end of the damped interval; None: from 10 Lanczos steps
    (``spectrum_upper_bound``, Section 3).  lam_f: its lower end (the cutoff);
    None: the largest Ritz value of the current block after each Rayleigh-Ritz
    step (the paper's alternative of a Lanczos estimate of the (n_b+1)-st
    eigenvalue, refined as the iteration proceeds), a number: fixed (the paper's
    0 for bound states).
    Each iteration filters the unlocked columns (degree - 1 products after the
    first step, which reuses H Q), projects them against the locked ones and
    orthonormalises them by CholeskyQR (twice), multiplies the new columns by H
    (one product: degree products per iteration in all), and solves
    T = Q^T H Q (the locked columns enter with their stored H Q and are rotated
    with the rest, as Section 3 describes).  Columns of the leading k whose
    relative residual is below tol are locked (lock=True) and not filtered.
    stop: optional callable(it, theta, rel_resid) -> bool (the hybrid switch,
    tested after the convergence test).  All n_b columns are returned in X, HX."""
    X0 = np.asarray(X0, dtype=np.float64)
    n, nb = X0.shape
    Q, _ = dense.cholqr(X0, passes=2)
    HQ = _apply(H, Q)
    spmm, spmv = 1, nb
    res = Result(None, None, None, None, 0, 0, 0, False)
    if lam_ub is None:
        lam_ub, _, _, _, m = spectrum_upper_bound(H, n, 10, X0[:, 0])
        spmm += m
        spmv += m
    theta, S = sla.eigh(0.5 * (Q.T @ HQ + HQ.T @ Q))
    Q, HQ = Q @ S, HQ @ S
    it = 0
    while True:
        R = HQ - Q * theta[None, :]
        rel = np.linalg.norm(R[:, :k], axis=0) / _scale(theta[:k], hnorm, norm)
        res.history.append(rel.copy())
        res.theta_hist.append(theta[:k].copy())
        if np.all(rel <= tol) or it >= maxiter:
            break
        if stop is not None and stop(it, theta, rel):
            res.events.append((it, "switch"))
            break
        it += 1
        locked = np.zeros(nb, dtype=bool)
        if lock:
            locked[:k] = rel <= tol
        act = ~locked
        lf = float(theta[-1]) if lam_f is None else float(lam_f)
        e = 0.5 * (lam_ub - lf)
        c = 0.5 * (lam_ub + lf)
        Y, p = cheb_filter(H, Q[:, act], HQ[:, act], degree, c, e)
        spmm += p
        spmv += p * int(act.sum())
        Ql, HQl = Q[:, locked], HQ[:, locked]
        for _ in range(2):
            Y = Y - Ql @ (Ql.T @ Y)
        Y = Y / np.linalg.norm(Y, axis=0)[None, :]
        Y, _ = dense.cholqr(Y, passes=2)
        HY = _apply(H, Y)
        spmm += 1
        spmv += int(act.sum())
        Qn = np.hstack([Ql, Y])
        HQn = np.hstack([HQl, HY])
        theta, S = sla.eigh(0.5 * (Qn.T @ HQn + HQn.T @ Qn))
        Q, HQ = Qn @ S, HQn @ S
    res.theta, res.X, res.HX = theta, Q, HQ
    res.resid = rel
    res.iters, res.spmm, res.spmv = it, spmm, spmv
    res.converged = bool(np.all(rel <= tol))
    res.events.append(("lambda_ub", lam_ub))
    return res


def merge_refined(state, Xr, H):
    """The hand-back after a LOBPCG front end (the project's reading; the paper
    has no hand-back): X becomes the n_b lowest Ritz vectors of span[X Xr],
    where Xr are RMM-DIIS's refined vectors.  Xr's part outside span[X] is
    taken by two classical Gram-Schmidt passes, columns whose remainder is
    below 1e-10 of their norm (no new direction) are dropped, the rest is
    orthonormalised by CholQR2 (Y), H Y is formed by one product, and a
    Rayleigh-Ritz step on [X Y]
    (eq. (rreig)) gives X and, by linearity, HX; P, HP, the locking state and
    the iteration count stay.  span[X] lies inside span[X Y] = span[X Xr], so no
    Ritz value rises (Courant-Fischer).  When Y cannot be orthonormalised (Xr
    adds no direction) the state stays as it is.  Returns (state, merged)."""
    X, HX = state["X"], state["HX"]
    nb = X.shape[1]
    Y = np.array(Xr, dtype=np.float64)
    before = np.linalg.norm(Y, axis=0)
    for _ in range(2):
        Y = Y - X @ (X.T @ Y)
    # a column whose part outside span[X] is at rounding level adds no direction
    keep = np.linalg.norm(Y, axis=0) > 1e-10 * before
    if not np.any(keep):
        return state, False
    try:
        Y, _ = dense.cholqr(Y[:, keep], passes=2)
    except dense.NotSPD:
        return state, False
    Z = np.hstack([X, Y])
    HZ = np.hstack([HX, H @ Y])
    try:
        theta, C = dense.rayleigh_ritz(Z.T @ HZ, Z.T @ Z, nb)
    except np.linalg.LinAlgError:
        return state, False
    new = dict(state)
    new["X"], new["HX"], new["theta"] = Z @ C, HZ @ C, theta
    return new, True


def hybrid(H, X0, k, front="lobpcg", switch="tau", switch_thr=1e-7, min_front=3, max_front=500,
           tol=1e-6, hnorm=1.0, norm="hnorm", d=None, s_max=10, rmm_maxiter=300, precond="jacobi",
           rmm_precond=None, fallback=True, max_back=2000, cheb_degree=10, nb_back=None):
    """Hybrid solver of Section 2.7 / Section 4: a block Lanczos, LOBPCG or
    ChebFSI front end, then batched RMM-DIIS on the leading k Ritz pairs.

    switch: "tau" (eq. (switchtau) below switch_thr, after at least min_front
    iterations), "resid" (largest relative residual of the leading k below
    switch_thr) or "iters" (exactly switch_thr front-end iterations).
    fallback: when RMM-DIIS stagnates (see ``rmm_diis(guard=True)``) or runs out
    of sweeps, LOBPCG takes over (the paper has no hand-back; this is the
    project's reading): after a LOBPCG front end it resumes that iteration from
    its state at the switch (RMM-DIIS works on copies), with X merged with the
    refined vectors by ``merge_refined`` unless they collapsed; after a block Lanczos
    or ChebFSI front end it starts (block nb_back, default the front end's
    block) from the refined vectors and the next Ritz vectors of the front end.
    A front end that reaches max_front hands over too (a fixed switch point).
    Returns (front, rmm, back) results; rmm and back are None when not
    reached; back.iters counts the iterations after the hand-back."""
    state = {"tprev": None}

    def stop(it, theta, rel):
        if switch == "iters":
            return it >= int(switch_thr)
        if switch == "resid":
            return bool(np.max(rel[:k]) < switch_thr) and it >= 1
        th = np.asarray(theta[:k])
        tprev = state["tprev"]
        state["tprev"] = th.copy()
        if tprev is None or it < min_front:
            return False
        return dense.switch_tau(th, tprev) < switch_thr

    nbb = np.asarray(X0).shape[1] if nb_back is None else nb_back
    if front == "lobpcg":
        fr = lobpcg(H, X0, k, tol=tol, maxiter=max_front, hnorm=hnorm, norm=norm, precond=precond, d=d,
                    stop=stop)
        Xk, HXk, Xrest = fr.X[:, :k], fr.HX[:, :k], None
    elif front == "chebfsi":
        fr = chebfsi(H, X0, k, degree=cheb_degree, tol=tol, maxiter=max_front, hnorm=hnorm, norm=norm, stop=stop)
        Xk, HXk, Xrest = fr.X[:, :k], fr.HX[:, :k], fr.X[:, k:nbb]
    else:
        fr = block_lanczos(H, X0, k, tol=tol, maxiter=max_front, hnorm=hnorm, norm=norm, stop=stop, nret=nbb)
        Xk, HXk, Xrest = fr.X[:, :k], fr.HX[:, :k], fr.X[:, k:nbb]
    if fr.converged:
        return fr, None, None
    rm = rmm_diis(H, Xk, k=k, HX=HXk, s_max=s_max, tol=tol, maxiter=rmm_maxiter, hnorm=hnorm,
                  norm=norm, precond=rmm_precond, guard=fallback)
    # converged columns that fell onto the same eigenpairs (RMM-DIIS refines
    # each column on its own; on clustered spectra several can reach one pair)
    # are not a result: the largest off-diagonal entry of their normalised Gram
    # matrix must be at most 1e-4, else the block is handed back as after a
    # stagnation (the project's reading; the paper notes the risk only)
    collapsed = False
    if rm.converged:
        Q = rm.X[:, :k] / np.linalg.norm(rm.X[:, :k], axis=0)[None, :]
        G = np.abs(Q.T @ Q - np.eye(k))
        collapsed = not (G.max() <= 1e-4)
        if collapsed:
            rm.events.append((rm.iters, "collapse"))
            rm.converged = False
    if rm.converged or not fallback:
        return fr, rm, None
    if front == "lobpcg":
        it0 = fr.state["it"]
        st, merged = fr.state, False
        if not collapsed:
            st, merged = merge_refined(st, rm.X[:, :k], H)
        back = lobpcg(H, None, k, tol=tol, maxiter=it0 + max_back, hnorm=hnorm, norm=norm, precond=precond, d=d,
                      state=st)
        back.iters -= it0
        back.events.insert(0, (0, "merged" if merged else "resumed"))
    else:
        Xb = fr.X[:, :nbb] if collapsed else np.hstack([rm.X[:, :k], Xrest])
        back = lobpcg(H, Xb, k, tol=tol, maxiter=max_back, hnorm=hnorm, norm=norm, precond=precond, d=d)
    return fr, rm, back


def final_check(H, X, hnorm):
    """Explicit FP64 check of returned pairs: theta_j = x^T H x / x^T x,
    ||H x - theta x|| / ||H||, ||H x - theta x|| / |theta| and ||X^T X - I||."""
    X = np.asarray(X, dtype=np.float64)
    HX = _apply(H, X)
    xx = np.einsum("ij,ij->j", X, X)
    theta = np.einsum("ij,ij->j", X, HX) / xx
    R = HX - X * theta[None, :]
    rn = np.linalg.norm(R, axis=0) / np.sqrt(xx)
    orth = np.linalg.norm(X.T @ X / np.sqrt(np.outer(xx, xx)) - np.eye(X.shape[1]))
    return theta, rn / hnorm, rn / np.abs(theta), orth


def lanczos_norm_estimate(H, n, steps=30, seed_vec=None):
    """||H||_2 estimate from a short single-vector Lanczos run (Section 2.1,
    with full re-orthogonalisation): returns (max |Ritz value|, the upper
    estimate theta_max + ||r_max|| used for lambda_ub in Section 3.2)."""
    v = np.ones(n) if seed_vec is None else np.asarray(seed_vec, dtype=np.float64)
    v = v / np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    w = None
    for j in range(steps):
        w = _apply(H, V[-1])
        a = V[-1] @ w
        w = w - a * V[-1] - (betas[-1] * V[-2] if betas else 0)
        Vm = np.array(V).T
        w = w - Vm @ (Vm.T @ w)
        b = np.linalg.norm(w)
        alphas.append(a)
        if b == 0 or j == steps - 1:
            betas.append(b)
            break
        betas.append(b)
        V.append(w / b)
    m = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:m - 1], 1) + np.diag(betas[:m - 1], -1)
    th, Q = np.linalg.eigh(T)
    low = max(abs(th[0]), abs(th[-1]))
    up = max(abs(th[0]) + betas[m - 1] * abs(Q[-1, 0]), abs(th[-1]) + betas[m - 1] * abs(Q[-1, -1]))
    return float(low), float(up)
