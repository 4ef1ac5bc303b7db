"""Pins for oracle.dense: identities, special cases, independent routes and
worked numbers from the paper."""
import os

import numpy as np
import pytest

import synthgen as sg
from oracle import dense

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_cholqr_identities():
    X = sg.normal_block(500, 8, 1)
    Q, R = dense.cholqr(X)
    np.testing.assert_allclose(Q.T @ Q, np.eye(8), atol=1e-12)
    np.testing.assert_allclose(Q @ R, X, atol=1e-12)
    assert np.allclose(R, np.triu(R)) and np.all(np.diag(R) > 0)
    Rh = np.linalg.qr(X)[1]
    np.testing.assert_allclose(R, np.diag(np.sign(np.diag(Rh))) @ Rh, atol=1e-10)


def test_cholqr2_repairs_ill_conditioned_block():
    X = sg.normal_block(2000, 6, 2)
    X[:, 5] = X[:, 4] + 1e-6 * X[:, 5]
    Q1, _ = dense.cholqr(X, passes=1)
    Q2, R2 = dense.cholqr(X, passes=2)
    e1 = np.linalg.norm(Q1.T @ Q1 - np.eye(6))
    e2 = np.linalg.norm(Q2.T @ Q2 - np.eye(6))
    assert e2 < 1e-13 and e2 < e1
    np.testing.assert_allclose(Q2 @ R2, X, atol=1e-10)


def test_cholqr_rank_deficient_raises():
    X = sg.normal_block(100, 3, 3)
    X[:, 2] = X[:, 0]
    with pytest.raises(dense.NotSPD):
        dense.cholqr(X)


def test_rayleigh_ritz_special_and_independent_route():
    # diagonal pencil: eigenvalues a_i / b_i
    a = np.array([3.0, -1.0, 2.0, 5.0])
    b = np.array([1.0, 2.0, 4.0, 0.5])
    th, C = dense.rayleigh_ritz(np.diag(a), np.diag(b), 2)
    np.testing.assert_allclose(th, np.sort(a / b)[:2])
    # general pencil: against L^{-1} A L^{-T} with L = cholesky(B)
    Z = sg.normal_block(12, 12, 4)
    A = Z + Z.T
    Y = sg.normal_block(30, 12, 5)
    B = Y.T @ Y
    th, C = dense.rayleigh_ritz(A, B, 5)
    L = np.linalg.cholesky(B)
    Li = np.linalg.inv(L)
    ref = np.linalg.eigvalsh(Li @ A @ Li.T)[:5]
    np.testing.assert_allclose(th, ref, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(C.T @ B @ C, np.eye(5), atol=1e-10)
    np.testing.assert_allclose(A @ C, B @ C * th[None, :], atol=1e-9)
    assert np.all(np.diff(th) >= 0)


def test_diis_against_substitution_form():
    rng = sg.normal_block(200, 5, 6)
    Bm = rng.T @ rng
    alpha = dense.diis_coefficients(Bm)
    assert abs(alpha.sum() - 1) < 1e-12
    # substitution form: alpha_last = 1 - sum(others); unconstrained least squares
    R = rng
    last = R[:, -1]
    D = R[:, :-1] - last[:, None]
    a_head = np.linalg.lstsq(D, -last, rcond=None)[0]
    ref = np.append(a_head, 1 - a_head.sum())
    np.testing.assert_allclose(alpha, ref, atol=1e-9)
    # optimality: combined residual is orthogonal to the differences
    rc = R @ alpha
    np.testing.assert_allclose(D.T @ rc, 0.0, atol=1e-9 * np.linalg.norm(R) ** 2)
    assert np.array_equal(dense.diis_coefficients(np.array([[2.5]])), np.ones(1))


def test_diis_singular_window():
    r = sg.normal_block(50, 1, 1)[:, 0]
    R = np.stack([r, r, 2 * r], axis=1)
    alpha = dense.diis_coefficients(R.T @ R)
    assert abs(alpha.sum() - 1) < 1e-9
    assert np.linalg.norm(R @ alpha) <= np.linalg.norm(r) * (1 + 1e-9)


def test_rr_2x2_closed_form():
    A = np.array([[1.0, 0.3], [0.3, 2.0]])
    B = np.array([[1.0, 0.2], [0.2, 0.5]])
    th, g = dense.rr_2x2(A, B)
    # det(A - t B) = 0  ->  (b00 b11 - b01^2) t^2 - (a00 b11 + a11 b00 - 2 a01 b01) t + det A = 0
    qa = B[0, 0] * B[1, 1] - B[0, 1] ** 2
    qb = -(A[0, 0] * B[1, 1] + A[1, 1] * B[0, 0] - 2 * A[0, 1] * B[0, 1])
    qc = A[0, 0] * A[1, 1] - A[0, 1] ** 2
    t_small = (-qb - np.sqrt(qb * qb - 4 * qa * qc)) / (2 * qa)
    assert abs(th - t_small) < 1e-13
    assert abs(g @ B @ g - 1) < 1e-13
    np.testing.assert_allclose(A @ g, th * (B @ g), atol=1e-13)


def test_switch_tau_worked_value():
    # theta^(k-1) = (1, 2), theta^(k) = (1.1, 2.2): each relative change is 1/11,
    # tau = (1/2) sqrt(2) / 11 (the 1/n_ev factor sits outside the root).
    tau = dense.switch_tau([1.1, 2.2], [1.0, 2.0])
    assert abs(tau - np.sqrt(2) / 22) < 1e-15
    assert dense.switch_tau([3.0, -4.0, 5.0], [3.0, -4.0, 5.0]) == 0.0


def test_effective_spmv_worked_example():
    kv = {}
    for line in open(os.path.join(GOLD, "effective_spmv_li6.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            kv[k] = float(v)
    ratio = kv["spmm_gflops"] / kv["spmv_gflops"]
    assert round(ratio, 1) == kv["ratio_printed"]
    eff = dense.effective_spmv(kv["iterations"] * kv["block_size"], kv["spmm_gflops"], kv["spmv_gflops"])
    assert round(eff) == kv["effective_printed"]
    assert eff < kv["lanczos_spmv"]


def test_rr_2x2_orientation():
    # the returned vector keeps a positive overlap with the first basis vector
    for A, B in [(np.array([[-4.0, 26.8], [26.8, 393.7]]), np.array([[1.0, 5e-8], [5e-8, 26.8]])),
                 (np.array([[1.0, -0.3], [-0.3, 2.0]]), np.eye(2))]:
        th, g = dense.rr_2x2(A, B)
        assert (B @ g)[0] > 0
