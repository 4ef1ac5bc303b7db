"""Pins for oracle.mlp: closed forms, finite differences, the MINRES optimality
property and the scaling relation between features, targets and the shifted
diagonal preconditioner."""
import numpy as np

import synthgen as sg
from oracle import mlp
from oracle import sparse as osp


def test_forward_closed_form():
    # hidden unit u < 4 passes feature u through the ReLU; w2 sums them
    p = np.zeros(mlp.NPARAM)
    W1 = np.zeros((64, 4))
    W1[np.arange(4), np.arange(4)] = 1.0
    p[:256] = W1.ravel()
    p[320:324] = 1.0
    p[384] = 0.5
    F = sg.normal_block(40, 4, 3)
    np.testing.assert_allclose(mlp.forward(p, F), np.maximum(F, 0).sum(axis=1) + 0.5, rtol=0, atol=1e-15)


def test_gradient_against_finite_differences():
    p = mlp.init_params(1)
    p[256:320] = 0.1 * sg.normal_block(64, 1, 4)[:, 0]
    F = sg.normal_block(50, 4, 5)
    t = sg.normal_block(50, 1, 6)[:, 0]
    L, g = mlp.loss_grad(p, F, t)
    assert abs(L - np.mean((mlp.forward(p, F) - t) ** 2)) < 1e-14
    h = 1e-6
    fd = np.empty(mlp.NPARAM)
    for q in range(mlp.NPARAM):
        e = np.zeros(mlp.NPARAM)
        e[q] = h
        fd[q] = (mlp.loss_grad(p + e, F, t)[0] - mlp.loss_grad(p - e, F, t)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_adam_first_step_and_quadratic():
    p0 = sg.normal_block(10, 1, 7)[:, 0]
    g = sg.normal_block(10, 1, 8)[:, 0]
    p1, m, v = mlp.adam_step(p0, g, np.zeros(10), np.zeros(10), 1, lr=1e-2)
    # bias-corrected moments of the first step are g and g^2
    np.testing.assert_allclose(p1, p0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-15)
    c = np.linspace(-1, 1, 10)
    p, m, v = np.zeros(10), np.zeros(10), np.zeros(10)
    for s in range(1, 3001):
        p, m, v = mlp.adam_step(p, 2 * (p - c), m, v, s, lr=1e-2)
    np.testing.assert_allclose(p, c, atol=1e-3)


def _sym_indefinite(n, seed):
    Z = sg.normal_block(n, n, seed)
    A = Z + Z.T
    return A


def test_minres_solves_in_n_steps_and_is_optimal():
    n = 12
    A = _sym_indefinite(n, 9)
    b = sg.normal_block(n, 1, 10)[:, 0]
    x, hist = mlp.minres(lambda v: A @ v, b, n)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-7, atol=1e-8)
    # the recurrence's residual estimate is the true residual, and it never grows
    for k in range(1, n):
        xk, hk = mlp.minres(lambda v: A @ v, b, k)
        assert abs(np.linalg.norm(b - A @ xk) - hk[-1]) < 1e-9 * np.linalg.norm(b)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))


def test_minres_minimises_over_the_krylov_space():
    # brute force: least-squares over span{b, Ab, ..., A^{k-1} b}
    n, k = 15, 5
    A = _sym_indefinite(n, 11)
    b = sg.normal_block(n, 1, 12)[:, 0]
    K = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(k)], axis=1)
    c = np.linalg.lstsq(A @ K, b, rcond=None)[0]
    x, _ = mlp.minres(lambda v: A @ v, b, k)
    np.testing.assert_allclose(x, K @ c, rtol=1e-6, atol=1e-8)


def test_correction_solutions_solve_the_projected_system():
    n = 40
    A = _sym_indefinite(n, 13)
    w, V = np.linalg.eigh(A)
    # Ritz block from a perturbed invariant subspace
    Q, _ = np.linalg.qr(V[:, :3] + 1e-2 * sg.normal_block(n, 3, 14))
    th, C = np.linalg.eigh(Q.T @ A @ Q)
    X = Q @ C
    R = A @ X - X * th
    T = mlp.correction_solutions(A, X, th, R, steps=n)
    P = np.eye(n) - X @ X.T
    for j in range(3):
        M = P @ (A - th[j] * np.eye(n)) @ P
        np.testing.assert_allclose(M @ T[:, j], -P @ R[:, j], atol=1e-8 * np.linalg.norm(R[:, j]))
        assert np.abs(X.T @ T[:, j]).max() < 1e-10 * np.linalg.norm(T[:, j])


def test_features_by_definition():
    spec = sg.MatrixSpec(96, 1, 3, 0.4, 31)
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSym(spec.n, rp, ci, v)
    D = H.dense()
    R = sg.normal_block(spec.n, 2, 15)
    theta = np.array([-1.5, 2.0])
    hn = np.linalg.norm(D, 2)
    F = mlp.features(np.diag(D), theta, R, np.abs(D).sum(axis=1), (D != 0).sum(axis=1), hn).reshape(spec.n, 2, 4)
    k, j = 17, 1
    assert abs(F[k, j, 0] - (D[k, k] - theta[j]) / hn) < 1e-15
    assert abs(F[k, j, 1] - R[k, j] / np.linalg.norm(R[:, j]) * np.sqrt(spec.n)) < 1e-13
    assert abs(F[k, j, 2] - np.abs(D[k]).sum() / hn) < 1e-14
    assert abs(F[k, j, 3] - np.count_nonzero(D[k]) / np.mean((D != 0).sum(axis=1))) < 1e-14
    # the oracle's row statistics of the half-stored form agree with the dense ones
    np.testing.assert_allclose(H.row_abs_sums(), np.abs(D).sum(axis=1), rtol=1e-14)
    np.testing.assert_array_equal(H.row_nnz(), (D != 0).sum(axis=1))


def test_shifted_diagonal_is_f1_over_f0():
    # the dimensionless target of the correction r / (d - theta) is exactly f1 / f0,
    # and an output equal to f1 / f0 reproduces the shifted diagonal
    n = 64
    d = np.linspace(-3, 5, n) + 0.01
    theta = np.array([-4.0, 6.0])
    R = sg.normal_block(n, 2, 16)
    hn = 7.5
    T = R / (d[:, None] - theta[None, :])
    F = mlp.features(d, theta, R, np.ones(n), np.ones(n), hn)
    tau = mlp.targets(T, R, hn)
    np.testing.assert_allclose(tau, F[:, 1] / F[:, 0], rtol=1e-12)
    rn = np.linalg.norm(R, axis=0)
    W = (F[:, 1] / F[:, 0]).reshape(n, 2) * rn / (hn * np.sqrt(n))
    np.testing.assert_allclose(W, T, rtol=1e-12)


def _apply_by_loops(p, R, theta, d, rowabs, rownnz, hnorm):
    """w_kj written out entry by entry: the four features, the 64 hidden units
    one at a time, the output, and the rescale by ||r_j|| / (||H|| sqrt(n))."""
    W1, b1, w2, b2 = mlp.unpack(p)
    n, ncol = R.shape
    mean_nz = sum(rownnz) / n
    out = np.zeros((n, ncol))
    for j in range(ncol):
        rn = np.sqrt(sum(R[k, j] ** 2 for k in range(n)))
        for k in range(n):
            f = [(d[k] - theta[j]) / hnorm, R[k, j] / rn * np.sqrt(n), rowabs[k] / hnorm, rownnz[k] / mean_nz]
            o = b2
            for h in range(mlp.NH):
                a = b1[h] + sum(W1[h, e] * f[e] for e in range(mlp.NF))
                o += w2[h] * max(a, 0.0)
            out[k, j] = o * rn / (hnorm * np.sqrt(n))
    return out


def test_precond_apply_by_definition():
    """The learned preconditioner's apply against its definition written out
    entry by entry, on a random network and a small residual block."""
    spec = sg.MatrixSpec(64, 1, 2, 0.4, 33)
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSym(spec.n, rp, ci, v)
    p = mlp.init_params(21)
    p[256:320] = 0.3 * sg.normal_block(64, 1, 22)[:, 0]
    p[384] = -0.2
    R = sg.normal_block(spec.n, 3, 23)
    theta = np.array([-2.0, 0.5, 3.0])
    hn = 11.0
    W = mlp.precond_apply(p, R, theta, H.d, H.row_abs_sums(), H.row_nnz(), hn)
    ref = _apply_by_loops(p, R, theta, H.d, H.row_abs_sums(), H.row_nnz(), hn)
    np.testing.assert_allclose(W, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_precond_apply_closed_forms():
    """Through precond_apply itself: (1) a network with out = f1 / f0 gives the
    shifted diagonal r_kj / (d_k - theta_j) of oracle.sparse.jacobi_apply
    (floor 0), which pins the rescale; (2) the ReLU network
    out = a relu(f1) - a relu(-f1) = a f1 gives w = a R / ||H||, whatever the
    other features; (3) a constant network out = c gives w_kj = c ||r_j|| /
    (||H|| sqrt(n))."""
    n = 80
    d = np.linspace(-3, 5, n) + 0.013
    theta = np.array([-4.0, 6.0, 9.5])
    R = sg.normal_block(n, 3, 24)
    rowabs = np.linspace(1.0, 2.0, n)
    rownnz = np.arange(n) % 7 + 1.0
    hn = 7.5
    W = mlp.precond_apply(None, R, theta, d, rowabs, rownnz, hn, net=lambda F: F[:, 1] / F[:, 0])
    np.testing.assert_allclose(W, osp.jacobi_apply(R, d, theta, 0.0) * np.sign(d[:, None] - theta[None, :]),
                               rtol=1e-12)
    np.testing.assert_allclose(W, R / (d[:, None] - theta[None, :]), rtol=1e-12)
    a = 0.37
    p = np.zeros(mlp.NPARAM)
    W1 = p[:256].reshape(64, 4)
    W1[0, 1], W1[1, 1] = 1.0, -1.0          # hidden 0 = relu(f1), hidden 1 = relu(-f1)
    p[320], p[321] = a, -a                  # out = a relu(f1) - a relu(-f1) = a f1
    W = mlp.precond_apply(p, R, theta, d, rowabs, rownnz, hn)
    np.testing.assert_allclose(W, a * R / hn, rtol=1e-12)
    q = np.zeros(mlp.NPARAM)
    q[384] = 1.25
    W = mlp.precond_apply(q, R, theta, d, rowabs, rownnz, hn)
    np.testing.assert_allclose(W, 1.25 * np.linalg.norm(R, axis=0)[None, :] / (hn * np.sqrt(n)) * np.ones((n, 1)),
                               rtol=1e-12)
