"""Pins for oracle.solvers: dense LAPACK eigh, closed-form spectra, planted
spectra with a degenerate cluster, and invariants of each method."""
import numpy as np
import pytest

import synthgen as sg
from oracle import dense, solvers
from oracle import sparse as osp


def _toeplitz(n, a=2.0, b=-1.0):
    rp = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        cols.append(i); vals.append(a)
        if i + 1 < n:
            cols.append(i + 1); vals.append(b)
        rp[i + 1] = len(cols)
    return osp.HalfSym(n, rp, np.array(cols, np.int32), np.array(vals, np.float32))


def _small(n=1024, seed=5):
    spec = sg.MatrixSpec(n, 6, 12, 0.25, seed)
    H = osp.HalfSym(n, *sg.gen_csr(spec))
    w = np.linalg.eigvalsh(H.dense())
    return spec, H, w


def _subspace_angle(X, Y):
    Qx = np.linalg.qr(X)[0]
    Qy = np.linalg.qr(Y)[0]
    # sine of the largest principal angle, from the projection residual
    return float(np.linalg.norm(Qy - Qx @ (Qx.T @ Qy), 2))


def test_lobpcg_closed_form_toeplitz():
    n = 60
    H = _toeplitz(n, 0.5, 1.0)
    # eigenvalues a + 2 b cos(k pi / (n + 1)), k = 1..n
    lam = np.sort(0.5 + 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    X0 = sg.normal_block(n, 6, 3)
    r = solvers.lobpcg(H, X0, 3, tol=1e-10, maxiter=2000, hnorm=2.5, d=H.d)
    assert r.converged
    np.testing.assert_allclose(r.theta[:3], lam[:3], rtol=1e-8, atol=1e-12)


def test_lobpcg_against_eigh_and_invariants():
    spec, H, w = _small()
    hn = np.max(np.abs(w))
    X0 = sg.start_block(spec, 8)
    r = solvers.lobpcg(H, X0, 6, tol=1e-7, maxiter=800, hnorm=hn, d=H.d)
    assert r.converged
    np.testing.assert_allclose(r.theta[:6], w[:6], rtol=1e-8)
    th = np.array(r.theta_hist)
    # Courant-Fischer: Ritz values never increase and stay above the eigenvalues
    assert np.all(np.diff(th, axis=0) <= 1e-9 * hn)
    assert np.all(th >= w[None, :6] - 1e-9 * hn)
    # recurrence-carried H X equals the explicit product
    np.testing.assert_allclose(r.HX, H @ r.X, atol=1e-9 * hn)
    thc, rh, rt, orth = solvers.final_check(H, r.X[:, :6], hn)
    assert np.all(rh <= 1e-7) and orth < 1e-10
    assert r.spmm == r.iters + 1


def test_block_lanczos_invariants_and_exactness():
    spec, H, w = _small(256, 9)
    hn = np.max(np.abs(w))
    X0 = sg.start_block(spec, 4)
    r = solvers.block_lanczos(H, X0, 4, tol=1e-10, maxiter=80, hnorm=hn)
    assert r.converged
    np.testing.assert_allclose(r.theta, w[:4], rtol=1e-9)
    # the Ritz residual estimate equals the explicit residual
    R = H @ r.X - r.X * r.theta[None, :]
    est = r.resid * hn
    np.testing.assert_allclose(np.linalg.norm(R, axis=0), est, atol=1e-9 * hn)
    np.testing.assert_allclose(r.HX, H @ r.X, atol=1e-8 * hn)
    # n_b = 1: block Lanczos reduces to Lanczos; after n steps the spectrum is exact
    n = 40
    Z = sg.normal_block(n, n, 1)
    A = Z + Z.T
    r1 = solvers.block_lanczos(A, np.ones((n, 1)), 1, tol=1e-13, maxiter=n, hnorm=np.abs(np.linalg.eigvalsh(A)).max())
    assert abs(r1.theta[0] - np.linalg.eigvalsh(A)[0]) < 1e-9


def _planted(n=300, seed=12):
    Q = np.linalg.qr(sg.normal_block(n, n, seed))[0]
    lam = np.concatenate([[-5.0, -4.0, -3.0, -2.0], np.linspace(0, 10, n - 4)])
    A = (Q * lam[None, :]) @ Q.T
    return 0.5 * (A + A.T), Q, lam


def test_rmm_diis_refines_ritz_quality_vectors():
    # start vectors with error only along the unwanted (higher) eigenvectors, the
    # situation after a Rayleigh-Ritz front end (Section 2.7)
    A, Q, lam = _planted()
    N = sg.normal_block(300, 4, 8)
    N -= Q[:, :4] @ (Q[:, :4].T @ N)
    X = Q[:, :4] + 1e-3 * N
    r = solvers.rmm_diis(A, X, k=4, s_max=10, tol=1e-10, maxiter=200, hnorm=10.0)
    assert r.converged and r.iters < 60
    np.testing.assert_allclose(r.theta, lam[:4], atol=1e-12)
    for j in range(4):
        assert _subspace_angle(r.X[:, [j]], Q[:, [j]]) < 1e-9
    np.testing.assert_allclose(r.HX, A @ r.X, atol=1e-12)


def test_rmm_diis_lowest_pair_from_any_nearby_start():
    A, Q, lam = _planted()
    X = Q[:, :1] + 1e-3 * sg.normal_block(300, 1, 8)
    r = solvers.rmm_diis(A, X, k=1, s_max=10, tol=1e-12, maxiter=200, hnorm=10.0)
    assert r.converged and abs(r.theta[0] - lam[0]) < 1e-13


def test_rmm_diis_first_sweep_lowers_theta():
    # x^(0) lies in span{x~, r~}, so the 2x2 Rayleigh-Ritz cannot raise theta
    spec, H, w = _small(512, 4)
    X = sg.normal_block(512, 4, 8)
    X0 = X / np.linalg.norm(X, axis=0)
    th0 = np.einsum("ij,ij->j", X0, H @ X0)
    r1 = solvers.rmm_diis(H, X, k=4, s_max=10, tol=0.0, maxiter=1, hnorm=1.0)
    assert np.all(r1.theta <= th0 + 1e-12) and np.all(r1.theta < th0)
    assert r1.spmm == 2  # H X0 and the batched H r~


def test_rmm_diis_residual_forms_reach_same_pairs():
    A, Q, lam = _planted()
    N = sg.normal_block(300, 3, 2)
    N -= Q[:, :3] @ (Q[:, :3].T @ N)
    X = Q[:, :3] + 1e-4 * N
    a = solvers.rmm_diis(A, X, s_max=6, tol=1e-10, hnorm=10.0)
    b = solvers.rmm_diis(A, X, s_max=6, tol=1e-10, hnorm=10.0, residual_form="sum")
    np.testing.assert_allclose(a.theta, lam[:3], atol=1e-12)
    np.testing.assert_allclose(b.theta, lam[:3], atol=1e-12)


@pytest.mark.parametrize("front", ["lobpcg", "blanczos", "chebfsi"])
def test_hybrid_against_eigh(front):
    spec, H, w = _small(1024, 6)
    hn = np.max(np.abs(w))
    X0 = sg.start_block(spec, 8)
    fr, rm, back = solvers.hybrid(H, X0, 5, front=front, switch="tau", switch_thr=1e-7, tol=1e-7, hnorm=hn,
                                  d=H.d, max_front=400)
    res = back if back is not None else (rm if rm is not None else fr)
    assert res.converged
    np.testing.assert_allclose(np.sort(res.theta[:5]), w[:5], rtol=1e-8)


def test_planted_spectrum_with_degenerate_cluster():
    n = 300
    Q = np.linalg.qr(sg.normal_block(n, n, 12))[0]
    lam = np.concatenate([[-5.0, -4.0, -4.0, -4.0 + 1e-9, -3.0], np.linspace(0, 10, n - 5)])
    A = (Q * lam[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    r = solvers.lobpcg(A, sg.normal_block(n, 8, 1), 5, tol=1e-9, maxiter=3000, hnorm=10.0,
                       d=np.diag(A).copy())
    assert r.converged
    np.testing.assert_allclose(r.theta[:5], lam[:5], atol=1e-8)
    # the cluster is only determined as a subspace
    assert _subspace_angle(r.X[:, 1:4], Q[:, 1:4]) < 1e-6


def test_switch_rules_fire():
    spec, H, w = _small(1024, 6)
    hn = np.max(np.abs(w))
    X0 = sg.start_block(spec, 8)
    fr, rm, back = solvers.hybrid(H, X0, 5, front="lobpcg", switch="iters", switch_thr=5, tol=1e-7, hnorm=hn,
                                  d=H.d)
    assert fr.iters == 5 and rm is not None
    assert (back if back is not None else rm).converged
    fr, rm, back = solvers.hybrid(H, X0, 5, front="lobpcg", switch="resid", switch_thr=1e-3, tol=1e-7, hnorm=hn,
                                  d=H.d)
    assert np.max(fr.history[-1]) < 1e-3 and np.max(fr.history[-2]) >= 1e-3


def test_norm_estimate_brackets_two_norm():
    spec, H, w = _small(512, 3)
    lo, up = solvers.lanczos_norm_estimate(H, 512, 30)
    hn = np.max(np.abs(w))
    assert lo <= hn * (1 + 1e-12) and lo > 0.9 * hn and up >= lo


def _golden_small_spectrum():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "small_n8192_seed100_spectrum.txt")
    kv = dict(l.split() for l in open(path) if l.strip() and not l.startswith("#"))
    lam = np.array([float(kv["lambda%d" % (i + 1)]) for i in range(32)])
    return lam, float(kv["norm2"])


def test_lobpcg_small_workload_against_dense_eigh():
    """n=8192, block 8, 8 pairs, shifted Jacobi, FP64, residual 1e-6 relative to
    ||H||_2; eigenvalues checked against dense LAPACK eigh."""
    lam, hn = _golden_small_spectrum()
    spec = sg.SMALL
    H = osp.HalfSym(spec.n, *sg.gen_csr(spec))
    r = solvers.lobpcg(H, sg.start_block(spec, 8), 8, tol=1e-6, maxiter=1000, hnorm=hn, d=H.d)
    assert r.converged
    np.testing.assert_allclose(r.theta[:8], lam[:8], rtol=1e-8)
    th, rh, rt, orth = solvers.final_check(H, r.X[:, :8], hn)
    assert np.all(rh <= 1e-6) and orth < 1e-10


# ---- ChebFSI (Alg. 3, Section 2.4) -------------------------------------------

@pytest.mark.parametrize("degree", [1, 2, 3, 10])
def test_cheb_filter_is_the_first_kind_polynomial(degree):
    """The filter equals V T_d((Lambda - c)/e) V^T X with T_d the first-kind
    Chebyshev polynomial evaluated by numpy (no recurrence): a doubled first
    step (second-kind U_d) or an off-by-one degree fails this."""
    n = 80
    G = sg.normal_block(n, n, 31)
    Qo, _ = np.linalg.qr(G)
    lam = np.linspace(-3.0, 9.0, n)
    H = (Qo * lam[None, :]) @ Qo.T
    X = sg.normal_block(n, 4, 32)
    c, e = 4.0, 4.5
    Y, prod = solvers.cheb_filter(H, X, H @ X, degree, c, e)
    coef = np.zeros(degree + 1)
    coef[degree] = 1.0
    ref = (Qo * np.polynomial.chebyshev.chebval((lam - c) / e, coef)[None, :]) @ (Qo.T @ X)
    assert prod == degree - 1
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_spectrum_upper_bound_residual_and_bound():
    """lambda_ub = theta + ||r|| with ||r|| from the Lanczos relation: equal to
    the explicit ||H u - theta u|| of the returned Ritz vector; theta is a
    Rayleigh quotient (<= lambda_max) and, with the top eigenvalue set apart,
    lambda_ub lies above lambda_max."""
    n = 200
    G = sg.normal_block(n, n, 33)
    Qo, _ = np.linalg.qr(G)
    lam = np.concatenate([np.linspace(-5.0, 5.0, n - 1), [12.0]])
    H = (Qo * lam[None, :]) @ Qo.T
    ub, theta, rn, u, m = solvers.spectrum_upper_bound(H, n, 10, sg.normal_block(n, 1, 34)[:, 0])
    assert m == 10
    assert abs(np.linalg.norm(u) - 1.0) < 1e-12
    assert abs(theta - u @ H @ u) < 1e-10
    assert abs(rn - np.linalg.norm(H @ u - theta * u)) < 1e-9
    assert theta <= lam.max() + 1e-12 and ub >= lam.max()


def test_chebfsi_against_eigh_and_product_count():
    _, H, w = _small()
    hn = float(np.abs(w).max())
    X0 = sg.normal_block(H.n, 8, 35)
    r = solvers.chebfsi(H, X0, 5, degree=10, tol=1e-6, maxiter=300, hnorm=hn)
    assert r.converged
    np.testing.assert_allclose(r.theta[:5], w[:5], rtol=1e-8)
    th, rh, _, orth = solvers.final_check(H, r.X[:, :5], hn)
    assert np.all(rh <= 1e-6) and orth < 1e-10
    # H Q0, 10 Lanczos steps, then degree products per iteration (locking only narrows them)
    assert r.spmm == 1 + 10 + 10 * r.iters
    assert r.spmv <= 8 + 10 + 10 * 8 * r.iters


def test_chebfsi_locking_and_fixed_cutoff():
    """Locking leaves converged columns unfiltered (fewer SpMVs, same pairs);
    the paper's fixed cutoff lambda_F = 0 (bound states) reaches the same pairs
    with more iterations on these spectra, which extend far above and below 0."""
    _, H, w = _small()
    hn = float(np.abs(w).max())
    X0 = sg.normal_block(H.n, 8, 36)
    a = solvers.chebfsi(H, X0, 5, degree=10, tol=1e-6, maxiter=300, hnorm=hn, lock=True)
    b = solvers.chebfsi(H, X0, 5, degree=10, tol=1e-6, maxiter=300, hnorm=hn, lock=False)
    f = solvers.chebfsi(H, X0, 5, degree=10, tol=1e-6, maxiter=400, hnorm=hn, lam_f=0.0)
    for r in (a, b, f):
        assert r.converged
        np.testing.assert_allclose(r.theta[:5], w[:5], rtol=1e-8)
    assert a.spmv <= b.spmv
    assert f.iters > a.iters


def test_lobpcg_resumed_run_equals_one_run():
    """Stopping LOBPCG at an iteration and continuing from its state gives the
    same iterates as one uninterrupted run (the hand-back after an RMM-DIIS
    stagnation resumes the front end this way)."""
    spec, H, w = _small(1024, 6)
    hn = np.max(np.abs(w))
    X0 = sg.start_block(spec, 8)
    one = solvers.lobpcg(H, X0, 5, tol=1e-8, maxiter=600, hnorm=hn, d=H.d)
    first = solvers.lobpcg(H, X0, 5, tol=1e-8, maxiter=600, hnorm=hn, d=H.d, stop=lambda it, th, rel: it >= 17)
    assert first.iters == 17 and not first.converged
    rest = solvers.lobpcg(H, None, 5, tol=1e-8, maxiter=600, hnorm=hn, d=H.d, state=first.state)
    assert rest.converged and rest.iters == one.iters
    np.testing.assert_array_equal(rest.theta, one.theta)
    np.testing.assert_array_equal(rest.X, one.X)
    hist = first.history[:-1] + rest.history
    assert len(hist) == len(one.history)
    for a, b in zip(hist, one.history):
        np.testing.assert_array_equal(a, b)


def test_rmm_diis_guard_fires_on_its_rules():
    """On the n=8192 matrix RMM-DIIS after a tau switch stops by its stagnation
    guard; recomputed from its per-sweep residual history, one of the three
    rules (10x above the best, no new best for 2 s_max sweeps, best not halved
    over the last s_max sweeps) holds at the sweep where it stopped and none
    held before."""
    spec = sg.SMALL
    H = osp.HalfSym(spec.n, *sg.gen_csr(spec))
    kv = dict(l.split() for l in open(__file__.replace("test_oracle_solvers.py", "golden/small_n8192_seed100_spectrum.txt"))
              if l.strip() and not l.startswith("#"))
    hn = float(kv["norm2"])
    tol, smax, k = 0.9e-6, 10, 5
    fr, rm, back = solvers.hybrid(H, sg.start_block(spec, 8), k, front="lobpcg", switch="tau", switch_thr=1e-7,
                                  tol=tol, hnorm=hn, d=H.d, s_max=smax, max_front=1000)
    assert rm is not None and not rm.converged and rm.events[-1][1] == "stagnation"
    hist = np.array(rm.history)          # row s: residuals after sweep s (row 0: the start)
    S = hist.shape[0] - 1
    done = np.zeros(k, dtype=bool)
    best = hist[0].copy()
    best_it = np.zeros(k, dtype=int)
    bests = []
    fired = []
    for s in range(1, S + 1):
        rel = hist[s]
        done |= rel <= tol
        imp = rel < best
        best = np.where(imp, rel, best)
        best_it = np.where(imp, s, best_it)
        bests.append(best.copy())
        bad = ~done & ((rel > 10 * best) | (s - best_it > 2 * smax))
        if len(bests) > smax:
            bad |= ~done & (best > 0.5 * bests[-1 - smax])
        fired.append(bool(bad.any()))
    assert fired[-1] and not any(fired[:-1])
    assert back is not None and back.converged


def test_rmm_diis_collapse_is_flagged():
    """An early fixed switch (2 LOBPCG iterations, 5 pairs, block 8) on the
    n=1024 matrix: RMM-DIIS without the guard drives columns onto the same
    eigenpair, every residual below the tolerance but wanted pairs missing.
    The hybrid flags the block as collapsed (not converged); with the guard and
    the hand-back it reaches the dense eigh pairs."""
    spec, H, w = _small(1024, 6)
    hn = np.max(np.abs(w))
    X0 = sg.normal_block(spec.n, 8, 101).astype(np.float32).astype(np.float64)
    fr, rm, back = solvers.hybrid(H, X0, 5, front="lobpcg", switch="iters", switch_thr=2, tol=0.9e-6, hnorm=hn,
                                  d=H.d, fallback=False, rmm_maxiter=300)
    assert back is None and not rm.converged and rm.events[-1][1] == "collapse"
    assert np.all(rm.resid[:5] <= 0.9e-6)                  # each column alone looks converged
    Q = rm.X[:, :5] / np.linalg.norm(rm.X[:, :5], axis=0)
    assert np.abs(Q.T @ Q - np.eye(5)).max() > 0.5          # but two of them are one pair
    assert np.abs(np.sort(rm.theta[:5]) - w[:5]).max() > 0.1
    fr, rm, back = solvers.hybrid(H, X0, 5, front="lobpcg", switch="iters", switch_thr=2, tol=0.9e-6, hnorm=hn,
                                  d=H.d, fallback=True, rmm_maxiter=300)
    assert back is not None and back.converged
    np.testing.assert_allclose(np.sort(back.theta[:5]), w[:5], rtol=1e-8)


def test_merge_refined_is_rayleigh_ritz_on_the_union():
    """The hand-back's merge (the project's reading): the n_b lowest Ritz pairs
    of span[X Xr].  Pinned against an independent route (an orthonormal basis
    of the span by QR, then a symmetric eigensolver), orthonormality, H X by a
    fresh product, Courant-Fischer (no Ritz value rises over X alone), and an
    Xr that adds no direction (zero, or inside span[X]) leaving the state as is."""
    rng = np.random.default_rng(17)
    n, nb, k = 200, 8, 5
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T) + np.diag(np.linspace(0.0, 20.0, n))
    X, _ = np.linalg.qr(rng.standard_normal((n, nb)))
    w0, V0 = np.linalg.eigh(X.T @ A @ X)
    X = X @ V0  # a Ritz basis, as LOBPCG holds it
    Xr = X[:, :k] + 0.1 * rng.standard_normal((n, k))
    P = rng.standard_normal((n, nb))
    state = {"X": X, "HX": A @ X, "P": P, "HP": A @ P, "theta": w0, "active": np.ones(nb, bool), "it": 7}
    new, merged = solvers.merge_refined(state, Xr, A)
    assert merged
    Xn = new["X"]
    assert np.abs(Xn.T @ Xn - np.eye(nb)).max() < 1e-12
    assert np.abs(new["HX"] - A @ Xn).max() < 1e-12 * np.abs(A).max() * n
    Q, _ = np.linalg.qr(np.hstack([X, Xr]))
    ref = np.linalg.eigvalsh(Q.T @ A @ Q)[:nb]
    np.testing.assert_allclose(new["theta"], ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(np.diag(Xn.T @ A @ Xn), new["theta"], rtol=0, atol=1e-11 * np.abs(ref).max())
    assert np.all(new["theta"] <= w0 + 1e-12 * np.abs(w0).max())
    assert new["P"] is P and new["it"] == 7
    same, merged0 = solvers.merge_refined(state, np.zeros((n, k)), A)
    assert not merged0 and same is state
    # Xr inside span[X] adds no direction: nothing to merge
    same, merged1 = solvers.merge_refined(state, X[:, :k] @ rng.standard_normal((k, k)), A)
    assert not merged1 and same is state
