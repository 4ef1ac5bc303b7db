"""Full-size checks at n = 2,097,152 (seed 101), in the launch configuration the
benchmark times (m = 16 FP32 columns, contiguous): sampled block rows of the
product against the oracle computed from the CSR band that reaches them, the
self-adjointness of the product, and the benchmark's hybrid solve in both forms:
final FP64 residual, and every eigenvalue within 1e-8 relative of the oracle's
reference spectrum (tests/golden/scale_n2097152_seed101_spectrum.txt, written
by make_c2_spectrum.py from two FP64 oracle routes to a residual of 1e-9).

Bound for the product: each output is an FP32 sum of at most L + 2 products
(L = full row length), so |y - y_exact| <= gamma_{L+2} (|H| |X|)_i with
gamma_k = k u / (1 - k u), u = 2^-24."""
import os

import numpy as np
import pytest

import synthgen as sg
from oracle import sparse as osp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "scale_n2097152_seed101_spectrum.txt")


def golden_lambdas(k):
    kv = dict(line.split() for line in open(GOLDEN) if line.strip() and not line.startswith("#"))
    return np.array([float(kv["lambda%d" % (i + 1)]) for i in range(k)])


@pytest.fixture(scope="module")
def hy():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_15552_amd import hyeig
    return hyeig


@pytest.fixture(scope="module")
def big(hy):
    spec = sg.SCALE
    rp, ci, v = sg.gen_csr(spec)
    ctx = hy.Context(0)
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v)
    rowlen = np.diff(rp)
    del rp, ci, v
    yield spec, ctx, M, rowlen
    M.close()
    ctx.close()


def test_product_sampled_block_rows(hy, big):
    spec, ctx, M, _ = big
    m = 16
    X = sg.normal_block(spec.n, m, 7).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    hy.spmm_sym(ctx, M, Xd, Yd)
    Y = Yd.cpu().numpy().astype(np.float64)
    assert np.isfinite(Y).all()
    Xf = X.astype(np.float64)
    for J in (0, 1, 4095, 4096, 33333, spec.nbr - 1):
        i0 = max(0, J - spec.w)
        brp, bci, bv = sg.gen_block_rows(spec, i0, J + 1)
        rows = np.arange(32 * J, min(32 * J + 32, spec.n))
        ref = osp.product_rows(spec.n, 32 * i0, brp, bci, bv, Xf, rows)
        mag = osp.product_rows(spec.n, 32 * i0, brp, bci, np.abs(bv), np.abs(Xf), rows)
        # full row lengths of the sampled rows (upper part + entries above in their columns)
        cnt = osp.product_rows(spec.n, 32 * i0, brp, bci, np.ones_like(bv), np.ones((spec.n, 1)), rows)[:, 0]
        k = cnt + 2
        gam = k * U32 / (1 - k * U32)
        err = np.abs(Y[rows] - ref)
        assert np.all(err <= gam[:, None] * mag + 1e-30), (J, float((err / (gam[:, None] * mag + 1e-30)).max()))


def test_product_self_adjoint_full_size(hy, big):
    spec, ctx, M, _ = big
    m = 16
    X = torch.from_numpy(sg.normal_block(spec.n, m, 11).astype(np.float32)).cuda()
    Z = torch.from_numpy(sg.normal_block(spec.n, m, 12).astype(np.float32)).cuda()
    HX = torch.empty_like(X)
    HZ = torch.empty_like(Z)
    hy.spmm_sym(ctx, M, X, HX)
    hy.spmm_sym(ctx, M, Z, HZ)
    a = (X.double() * HZ.double()).sum(dim=0)
    b = (HX.double() * Z.double()).sum(dim=0)
    scale = (X.double().abs() * HZ.double().abs()).sum(dim=0)
    # each of the two FP32 products carries at most gamma_{L+2} relative error per entry (L <= 600 here)
    bound = 2 * 602 * U32 * scale * 10
    assert torch.all((a - b).abs() <= bound), ((a - b).abs() / scale).max().item()


def test_benchmark_solve_full_size(hy, big):
    spec, ctx, M, _ = big
    X0 = torch.from_numpy(sg.start_block(spec, 16).astype(np.float32)).cuda()
    p = hy.params_default(k=1, nb=1, method=hy.LOBPCG, tol=1.0, hnorm=0.0, maxiter=0)
    _, _, rep0, _, _ = hy.solve_lowest_k(ctx, M, p, X0[:, :1].clone())
    hn = rep0.hnorm_used
    out = {}
    for prec in (hy.PREC_F32, hy.PREC_PLAIN_F64):
        p = hy.params_default(k=10, nb=16, method=hy.LOBPCG_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=2000,
                              switch_rule=hy.SWITCH_RESID, switch_thr=1e-3, s_max=10, rmm_maxiter=300,
                              precision=prec, precond=hy.PRECOND_JACOBI)
        X = X0.clone()
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
        assert st == hy.OK, (prec, st)
        # the final check is an explicit FP64-accumulated product on the returned vectors
        assert rs.max() <= 1e-6, (prec, rs.max())
        assert rep.orth_err < 1e-5
        out[prec] = ev
    rel = np.abs(out[hy.PREC_F32] - out[hy.PREC_PLAIN_F64]) / np.abs(out[hy.PREC_PLAIN_F64])
    assert rel.max() < 1e-8, rel
    assert np.all(np.diff(out[hy.PREC_PLAIN_F64]) >= 0)
    lam = golden_lambdas(10)
    for prec, ev in out.items():
        err = np.abs(np.asarray(ev) - lam) / np.abs(lam)
        print("\nform %d: max relative eigenvalue error against the oracle's reference %.2e" % (prec, err.max()))
        assert err.max() <= 1e-8, (prec, err)
