"""Checks at n = 33,554,432 (seed 102): 1,048,576 block rows with 48 upper
tiles each inside a band of 16384 block rows, p = 0.25, about 1.3e10 stored
entries (past 2^31) and a 120 GB prepared matrix.

- the product at the block Lanczos width (m = 8, FP32, the tile walk) and at
  the LOBPCG width (m = 16, the matrix-core kernel): sampled block rows
  against the oracle, with the bound of the full-size check at n = 2,097,152;
- the FP64-accumulated form the final check uses and the plain FP64 form
  (FP64 x), on the same rows;
- self-adjointness of the product;
- block Lanczos (n_b = 8) -> RMM-DIIS for the 8 lowest pairs (LOBPCG with 16
  columns if RMM-DIIS stagnates): the final FP64 residual and orthonormality
  the library reports, and sampled rows of the residual recomputed by the
  oracle from the generator.

The oracle's rows of H X for block row J need the upper-triangle rows of J and
of the block rows whose tiles reach block column J (the generator names them:
about 48 of the 16384 before J); the rows of every other block row of the band
hold no entry in J's columns and are left empty.

Generating the matrix takes about a minute on 16 host threads and preparing it
about 225 GB of device memory at its peak (the tests skip on a device with
less than 280 GB); the four tests take about two minutes in all."""
import sys

import numpy as np
import pytest

import synthgen as sg
from oracle import sparse as osp

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _log(msg):
    print(msg, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def hy():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if torch.cuda.mem_get_info()[1] < 280e9:
        pytest.skip("needs a device with at least 280 GB")
    from paper_2305_15552_amd import hyeig
    return hyeig


@pytest.fixture(scope="module")
def large(hy):
    spec = sg.LARGE
    torch.cuda.empty_cache()
    rp, ci, v, nnz = sg.device_csr(spec, "cuda:0", chunk=65536, log=_log)
    ctx = hy.Context(0)
    M = hy.Matrix(ctx, spec.n, rp, ci, v, nnz=nnz)
    torch.cuda.synchronize()
    del rp, ci, v
    torch.cuda.empty_cache()
    _log("large: prepared %d tiles, %.1f GB" % (M.info.ntiles, M.info.prepared_bytes / 1e9))
    yield spec, ctx, M, nnz
    M.close()
    ctx.close()
    torch.cuda.empty_cache()


def _reaching_band(spec, J):
    """CSR rows 32 i0 .. 32 (J + 1) - 1 (i0 = max(0, J - w)) holding the
    upper-triangle rows of block row J and of every block row whose tiles reach
    block column J; all other rows empty.  Returns (row0, rowptr, colidx, vals)."""
    i0 = max(0, J - spec.w)
    src = [I for I in range(i0, J) if J in sg.tile_cols(spec, I)] + [J]
    nloc = 32 * (J + 1 - i0) if J + 1 < spec.nbr else spec.n - 32 * i0
    counts = np.zeros(nloc + 1, dtype=np.int64)
    parts = []
    for I in src:
        brp, bci, bv = sg.gen_block_rows(spec, I, I + 1)
        r0 = 32 * (I - i0)
        counts[r0 + 1:r0 + 1 + brp.size - 1] = np.diff(brp)
        parts.append((bci, bv))
    rowptr = np.cumsum(counts)
    colidx = np.concatenate([p[0] for p in parts])
    vals = np.concatenate([p[1] for p in parts])
    return 32 * i0, rowptr, colidx, vals


SAMPLES = (0, 1, 16383, 16384, 524287, 1048575)


@pytest.mark.parametrize("m", [8, 16])
def test_large_product_sampled_block_rows(hy, large, m):
    spec, ctx, M, _ = large
    X = sg.normal_block(spec.n, m, 7)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    Yd = torch.empty_like(Xd)
    hy.spmm_sym(ctx, M, Xd, Yd)
    Y64 = torch.empty((spec.n, m), dtype=torch.float64, device="cuda")
    hy.spmm_sym(ctx, M, Xd, Y64)  # FP64 accumulation of the FP32 data (the final check's form)
    Y = Yd.cpu().numpy().astype(np.float64)
    Yw = Y64.cpu().numpy()
    del Yd
    # the plain FP64 form: FP64 x, FP64 sums
    X64d = torch.from_numpy(X).cuda()
    hy.spmm_sym(ctx, M, X64d, Y64)
    Yp = Y64.cpu().numpy()
    del Y64, X64d
    torch.cuda.empty_cache()
    assert np.isfinite(Y).all() and np.isfinite(Yw).all() and np.isfinite(Yp).all()
    Xf = X.astype(np.float32).astype(np.float64)
    for J in SAMPLES:
        row0, brp, bci, bv = _reaching_band(spec, J)
        rows = np.arange(32 * J, min(32 * J + 32, spec.n))
        ref = osp.product_rows(spec.n, row0, brp, bci, bv, Xf, rows)
        mag = osp.product_rows(spec.n, row0, brp, bci, np.abs(bv), np.abs(Xf), rows)
        cnt = osp.product_rows(spec.n, row0, brp, bci, np.ones_like(bv), np.ones((spec.n, 1)), rows)[:, 0]
        assert cnt.min() > 300, (J, cnt.min())  # the rows are the band's full rows, not a truncated part
        k = cnt + 2
        gam = k * U32 / (1 - k * U32)
        err = np.abs(Y[rows] - ref)
        assert np.all(err <= gam[:, None] * mag + 1e-30), (J, float((err / (gam[:, None] * mag + 1e-30)).max()))
        # FP32 x FP32 products are exact in FP64; only the FP64 sums round
        gam64 = k * U64 / (1 - k * U64)
        err64 = np.abs(Yw[rows] - ref)
        assert np.all(err64 <= gam64[:, None] * mag + 1e-300), (J, float((err64 / (gam64[:, None] * mag)).max()))
        # FP64 x: each product rounds once more (k counts it)
        refp = osp.product_rows(spec.n, row0, brp, bci, bv, X, rows)
        magp = osp.product_rows(spec.n, row0, brp, bci, np.abs(bv), np.abs(X), rows)
        errp = np.abs(Yp[rows] - refp)
        assert np.all(errp <= gam64[:, None] * magp + 1e-300), (J, float((errp / (gam64[:, None] * magp)).max()))


def test_large_product_self_adjoint(hy, large):
    spec, ctx, M, _ = large
    m = 8
    X = torch.from_numpy(sg.normal_block(spec.n, m, 11).astype(np.float32)).cuda()
    Z = torch.from_numpy(sg.normal_block(spec.n, m, 12).astype(np.float32)).cuda()
    HX = torch.empty_like(X)
    HZ = torch.empty_like(Z)
    hy.spmm_sym(ctx, M, X, HX)
    hy.spmm_sym(ctx, M, Z, HZ)
    a = (X.double() * HZ.double()).sum(dim=0)
    b = (HX.double() * Z.double()).sum(dim=0)
    scale = (X.double().abs() * HZ.double().abs()).sum(dim=0)
    # rows hold at most ~900 entries here: gamma_{L+2} relative error per entry of each product
    bound = 2 * 902 * U32 * scale * 10
    assert torch.all((a - b).abs() <= bound), ((a - b).abs() / scale).max().item()
    del X, Z, HX, HZ
    torch.cuda.empty_cache()


def test_large_block_lanczos_rmm_diis(hy, large):
    spec, ctx, M, _ = large
    X0 = torch.from_numpy(sg.start_block(spec, 8).astype(np.float32)).cuda()
    p = hy.params_default(k=8, nb=8, method=hy.BLANCZOS_RMMDIIS, tol=1e-6, hnorm=0.0, maxiter=40,
                          switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, s_max=10, rmm_maxiter=200,
                          nb_back=16, maxiter_back=1500, precision=hy.PREC_F32, precond=hy.PRECOND_JACOBI)
    X = X0.clone()
    ev, rs, rep, st, hist = hy.solve_lowest_k(ctx, M, p, X, hist_cap=4000)
    _log("large solve: status %d, front %d rmm %d back %d, %.1f s, max resid %.2e" % (
        st, rep.iters_front, rep.iters_rmm, rep.iters_back, rep.ms_total / 1e3, rs.max()))
    assert st == hy.OK, (st, rs)
    assert rs.max() <= 1e-6 and rep.orth_err < 1e-5
    assert np.all(np.diff(ev) >= 0)
    # residual rows recomputed by the oracle: the squares over the sampled rows
    # cannot exceed the library's whole-vector residual
    Xh = X[:, :8].cpu().numpy().astype(np.float64)
    ss = np.zeros(8)
    for J in SAMPLES:
        row0, brp, bci, bv = _reaching_band(spec, J)
        rows = np.arange(32 * J, min(32 * J + 32, spec.n))
        HXr = osp.product_rows(spec.n, row0, brp, bci, bv, Xh, rows)
        ss += ((HXr - Xh[rows] * ev[None, :]) ** 2).sum(axis=0)
    hn = rep.hnorm_used
    assert np.all(np.sqrt(ss) <= rs * hn * 1.01 + 1e-12), (np.sqrt(ss), rs * hn)
