"""Chebyshev-filtered subspace iteration (Alg. 3) on the GPU through the C-ABI,
against the FP64 oracle (same start block, same lambda_ub from 10 Lanczos
steps on the first column) and against dense eigh."""
import os

import numpy as np
import pytest

import synthgen as sg
from oracle import solvers
from oracle import sparse as osp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "small_n8192_seed100_spectrum.txt")


@pytest.fixture(scope="module")
def hy():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_15552_amd import hyeig
    return hyeig


@pytest.fixture(scope="module")
def ctx(hy):
    c = hy.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def mid(hy, ctx):
    spec = sg.MatrixSpec(1024, 6, 12, 0.25, 6)
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSym(spec.n, rp, ci, v)
    w = np.linalg.eigvalsh(H.dense())
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v)
    return spec, H, M, w


def test_chebfsi_against_eigh_and_oracle(hy, ctx, mid):
    """5 pairs, block 8, degree 10, plain FP64 form: eigenvalues within 1e-8 of
    dense eigh, the oracle's iteration count, and degree products per
    iteration after H Q0 and the 10 Lanczos steps."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, 8).astype(np.float32)
    p = hy.params_default(k=5, nb=8, method=hy.CHEBFSI, tol=1e-6, hnorm=hn, maxiter=200, cheb_degree=10,
                          precision=hy.PREC_PLAIN_F64)
    X = torch.from_numpy(X0.copy()).cuda()
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.OK, (rep.iters_front, rs)
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    assert np.all(rs <= 1e-6)
    ref = solvers.chebfsi(H, X0.astype(np.float64), 5, degree=10, tol=0.9e-6, maxiter=200, hnorm=hn)
    assert ref.converged and abs(rep.iters_front - ref.iters) <= 1, (rep.iters_front, ref.iters)
    # + the final FP64 check's product
    assert rep.spmm_count == 1 + 10 + 10 * rep.iters_front + 1
    th, rh, _, orth = solvers.final_check(H, X[:, :5].cpu().numpy().astype(np.float64), hn)
    np.testing.assert_allclose(th, ev, rtol=1e-12)
    assert np.all(rh <= 1e-6)


@pytest.mark.parametrize("iters", [1, 3])
def test_chebfsi_step_parity(hy, ctx, mid, iters):
    """The same number of filtered iterations from the same start block: the
    FP64 GPU path and the oracle reach the same Ritz values."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, 8).astype(np.float32)
    p = hy.params_default(k=5, nb=8, method=hy.CHEBFSI, tol=1e-14, hnorm=hn, maxiter=iters, cheb_degree=6,
                          precision=hy.PREC_PLAIN_F64)
    X = torch.from_numpy(X0.copy()).cuda()
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.ENOCONV and rep.iters_front == iters
    ref = solvers.chebfsi(H, X0.astype(np.float64), 5, degree=6, tol=1e-14, maxiter=iters, hnorm=hn)
    # returned vectors are FP32: the Rayleigh quotient moves by about 2 u32 ||r|| ||H||
    bound = 4 * 2.0 ** -24 * rs * hn + 1e-11 * np.abs(ev)
    assert np.all(np.abs(ev - ref.theta[:5]) <= bound), (ev, ref.theta)


def test_chebfsi_fp32_small_workload_and_fixed_cutoff(hy, ctx):
    """FP32 form on the n = 8192 matrix, 8 pairs with block 16: eigenvalues
    within 1e-8 of the dense-eigh spectrum; the paper's fixed cutoff
    lambda_F = 0 reaches the same pairs."""
    kv = dict(l.split() for l in open(GOLD) if l.strip() and not l.startswith("#"))
    lam = np.array([float(kv["lambda%d" % (i + 1)]) for i in range(8)])
    hn = float(kv["norm2"])
    spec = sg.SMALL
    rp, ci, v = sg.gen_csr(spec)
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v)
    X0 = torch.from_numpy(sg.start_block(spec, 16).astype(np.float32)).cuda()
    its = {}
    for fixed in (0, 1):
        p = hy.params_default(k=8, nb=16, method=hy.CHEBFSI, tol=1e-6, hnorm=hn, maxiter=600, cheb_degree=10,
                              cheb_fixed_cutoff=fixed, cheb_cutoff=0.0, precision=hy.PREC_F32)
        X = X0.clone()
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
        assert st == hy.OK, (fixed, rep.iters_front, rs)
        np.testing.assert_allclose(ev, lam, rtol=1e-8)
        assert np.all(rs <= 1e-6)
        its[fixed] = rep.iters_front
    print("\nChebFSI n=8192, 8 pairs, block 16, degree 10: %d iterations (adaptive cutoff), %d (cutoff 0)"
          % (its[0], its[1]))
    M.close()


def test_chebfsi_rmm_diis_hybrid(hy, ctx, mid):
    """ChebFSI front end -> RMM-DIIS (tau < 1e-7 switch), LOBPCG if RMM-DIIS
    stagnates: the pairs against dense eigh, the switch and the front-end
    iteration count against the oracle's hybrid."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, 8).astype(np.float32)
    p = hy.params_default(k=5, nb=8, method=hy.CHEBFSI_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=200,
                          switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, s_max=10, rmm_maxiter=300,
                          cheb_degree=10, precision=hy.PREC_PLAIN_F64)
    X = torch.from_numpy(X0.copy()).cuda()
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    print("\nChebFSI -> RMM-DIIS: front %d, RMM-DIIS %d, LOBPCG %d, switched %d, fallback %d"
          % (rep.iters_front, rep.iters_rmm, rep.iters_back, rep.switched, rep.fallback_used))
    assert st == hy.OK and rep.switched == 1
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    assert np.all(rs <= 1e-6)
    fr, rm, back = solvers.hybrid(H, X0.astype(np.float64), 5, front="chebfsi", switch="tau", switch_thr=1e-7,
                                  tol=0.9e-6, hnorm=hn, d=H.d, max_front=200)
    assert abs(rep.iters_front - fr.iters) <= 1, (rep.iters_front, fr.iters)


def test_chebfsi_argument_errors(hy, ctx, mid):
    spec, H, M, w = mid
    X = torch.from_numpy(sg.start_block(spec, 8).astype(np.float32)).cuda()
    for kw in (dict(cheb_degree=0), dict(cheb_upper=-1.0)):
        with pytest.raises(hy.HyeigError) as e:
            hy.solve_lowest_k(ctx, M, hy.params_default(k=5, nb=8, method=hy.CHEBFSI, hnorm=30.0, **kw), X)
        assert e.value.status == hy.EINVAL
