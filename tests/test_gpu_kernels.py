"""GPU parity of the hot-path kernels against the FP64 oracle, called through
the C-ABI.  Floating-point tolerances follow the standard summation bound
|fl(sum) - sum| <= gamma_K sum|terms|, gamma_K = K u / (1 - K u), with K the
number of terms and u the unit roundoff of the accumulation type."""
import math

import numpy as np
import pytest

import synthgen as sg
from oracle import sparse as osp
from oracle import dense as odense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _gamma(K, u):
    return K * u / (1 - K * u)


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


MATS = {
    "ragged_n1000": sg.MatrixSpec(1000, 5, 8, 0.3, 21),
    "ragged_n4113": sg.MatrixSpec(4113, 7, 20, 0.25, 22),
    "small_n8192": sg.SMALL,
    "dense_tiles": sg.MatrixSpec(640, 19, 19, 0.9, 23),
}


@pytest.fixture(scope="module")
def mats(hy, ctx):
    out = {}
    for name, spec in MATS.items():
        rp, ci, v = sg.gen_csr(spec)
        H = osp.HalfSym(spec.n, rp, ci, v)
        M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v, flags=hy.MAT_VALIDATE | hy.MAT_BF16 | hy.MAT_ROWSTATS)
        out[name] = (spec, H, M)
    return out


def _bound(H, X, u):
    absH = abs(H.U) + abs(H.U.T) - osp.sp.diags(np.abs(H.d))
    K = np.asarray((absH != 0).sum(axis=1)).ravel()[:, None] + 1
    return _gamma(K, u) * (absH @ np.abs(X)) + 1e-300


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("m", [1, 3, 8, 9, 10, 11, 12, 15, 16, 32])
def test_spmm_fp32_against_oracle(hy, ctx, mats, name, m):
    # widths 9-16 run on matrix cores, the others walk the tiles; "dense_tiles"
    # (90% full tiles) takes the matrix-core kernel's path for tiles over 512 entries
    spec, H, M = mats[name]
    X = sg.normal_block(spec.n, m, 5).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.full((spec.n, m), float("nan"), dtype=torch.float32, device="cuda")
    hy.spmm_sym(ctx, M, Xd, Yd)
    Y = Yd.cpu().numpy().astype(np.float64)
    ref = H @ X.astype(np.float64)
    err = np.abs(Y - ref)
    assert np.all(err <= _bound(H, X.astype(np.float64), U32) + 1e-30)


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("m", [1, 8, 9, 12, 15, 16])
def test_spmm_fp64_and_mixed_against_oracle(hy, ctx, mats, name, m):
    # FP64 sums: widths 9-16 on FP64 matrix cores (dense 32 x 32 tiles, exact
    # zeros for the absent entries), narrower ones walk the tiles
    spec, H, M = mats[name]
    X = sg.normal_block(spec.n, m, 6)
    ref = H @ X
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty((spec.n, m), dtype=torch.float64, device="cuda")
    hy.spmm_sym(ctx, M, Xd, Yd)
    assert np.all(np.abs(Yd.cpu().numpy() - ref) <= _bound(H, X, U64))
    # FP32 X, FP64 accumulation: exact products of FP32 numbers summed in FP64
    X32 = X.astype(np.float32)
    ref32 = H @ X32.astype(np.float64)
    hy.spmm_sym(ctx, M, torch.from_numpy(X32).cuda(), Yd)
    assert np.all(np.abs(Yd.cpu().numpy() - ref32) <= _bound(H, X32.astype(np.float64), U64))


@pytest.mark.parametrize("m", [8, 16])
def test_spmm_bf16_values(hy, ctx, mats, m):
    # BF16 values take the tile walk at every width (16: the LOBPCG block)
    spec, H, M = mats["small_n8192"]
    # oracle on the BF16-rounded values (round to nearest even)
    rp, ci, v = sg.gen_csr(spec)
    vb = v.view(np.uint32).astype(np.uint64)
    vb = ((vb + 0x7FFF + ((vb >> 16) & 1)) >> 16) << 16
    v16 = vb.astype(np.uint32).view(np.float32)
    Hb = osp.HalfSym(spec.n, rp, ci, v16)
    X = sg.normal_block(spec.n, m, 7).astype(np.float32)
    Yd = torch.empty((spec.n, m), dtype=torch.float32, device="cuda")
    hy.spmm_sym(ctx, M, torch.from_numpy(X).cuda(), Yd, vdt=hy.BF16)
    ref = Hb @ X.astype(np.float64)
    assert np.all(np.abs(Yd.cpu().numpy() - ref) <= _bound(Hb, X.astype(np.float64), U32))


def test_spmm_ld_strided_and_self_adjoint(hy, ctx, mats):
    spec, H, M = mats["ragged_n4113"]
    big = torch.from_numpy(sg.normal_block(spec.n, 48, 8)).cuda()
    X = big[:, 16:32]             # column slice, ld = 48
    Yfull = torch.zeros((spec.n, 40), dtype=torch.float64, device="cuda")
    Y = Yfull[:, 8:24]
    hy.spmm_sym(ctx, M, X, Y)
    ref = H @ X.cpu().numpy()
    assert np.all(np.abs(Y.cpu().numpy() - ref) <= _bound(H, X.cpu().numpy(), U64))
    assert torch.all(Yfull[:, :8] == 0) and torch.all(Yfull[:, 24:] == 0)
    Z = torch.from_numpy(sg.normal_block(spec.n, 16, 9)).cuda()
    HZ = torch.empty_like(Z)
    hy.spmm_sym(ctx, M, Z, HZ)
    lhs = float((X * HZ).sum())
    rhs = float((Y * Z).sum())
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_spmv_on_a_strided_column(hy, ctx, mats):
    """One column of an n x 10 FP32 block multiplied alone (the decoupled
    RMM-DIIS product): it matches the oracle under the FP32 bound, touches no
    other column of the output, and agrees with that column of the 10-wide
    product (the same sums in the same order: printed whether bit for bit)."""
    spec, H, M = mats["ragged_n4113"]
    n, k, j = spec.n, 10, 7
    X = torch.from_numpy(sg.normal_block(n, k, 12).astype(np.float32)).cuda()
    Yb = torch.empty_like(X)
    hy.spmm_sym(ctx, M, X, Yb)
    Yc = torch.full_like(X, float("nan"))
    hy.spmm_sym(ctx, M, X[:, j:j + 1], Yc[:, j:j + 1])
    col = Yc[:, j].cpu().numpy().astype(np.float64)
    x = X[:, j].cpu().numpy().astype(np.float64)[:, None]
    ref = (H @ x)[:, 0]
    assert np.all(np.abs(col - ref) <= _bound(H, x, U32)[:, 0] + 1e-30)
    others = torch.cat([Yc[:, :j], Yc[:, j + 1:]], dim=1)
    assert torch.isnan(others).all()
    same = bool(torch.equal(Yc[:, j], Yb[:, j]))
    print("\nSpMV on column %d vs the same column of the 10-wide product: %s" % (j, "bitwise equal" if same else
          "max difference %.3g" % float((Yc[:, j] - Yb[:, j]).abs().max())))
    assert np.all(np.abs(col - Yb[:, j].cpu().numpy()) <= 2 * _bound(H, x, U32)[:, 0] + 1e-30)


@pytest.mark.parametrize("m,ldx,off", [(3, 16, 0), (10, 16, 0), (13, 16, 0), (10, 20, 4), (6, 8, 0), (20, 24, 0),
                                        (20, 20, 4), (12, 16, 4), (8, 12, 0)])
def test_spmm_partial_columns_in_wide_rows(hy, ctx, mats, m, ldx, off):
    # m columns inside rows of stride ldx, NaN in every other element of the
    # buffer, which ends at the last element of the last row (the product reads
    # 16-byte pieces when m columns end on a piece boundary, past column m
    # inside the stride, and single elements otherwise)
    spec, H, M = mats["ragged_n4113"]
    n = spec.n
    X = sg.normal_block(n, m, 10).astype(np.float32)
    flat = torch.full(((n - 1) * ldx + off + m,), float("nan"), dtype=torch.float32, device="cuda")
    Xd = flat.as_strided((n, m), (ldx, 1), off)
    Xd.copy_(torch.from_numpy(X).cuda())
    Yd = torch.full((n, m), float("nan"), dtype=torch.float32, device="cuda")
    hy.spmm_sym(ctx, M, Xd, Yd)
    Y = Yd.cpu().numpy().astype(np.float64)
    ref = H @ X.astype(np.float64)
    assert np.isfinite(Y).all()
    assert np.all(np.abs(Y - ref) <= _bound(H, X.astype(np.float64), U32) + 1e-30)


def test_matrix_stats(hy, ctx, mats):
    spec, H, M = mats["ragged_n4113"]
    np.testing.assert_array_equal(M.diag().cpu().numpy(), H.d.astype(np.float32))
    np.testing.assert_allclose(M.rowabs().cpu().numpy(), H.row_abs_sums(), rtol=1e-5)
    np.testing.assert_array_equal(M.rownnz().cpu().numpy(), H.row_nnz().astype(np.float32))


def test_matrix_validation_rejects_lower_entries(hy, ctx):
    rp = torch.tensor([0, 2, 3], dtype=torch.int64, device="cuda")
    ci = torch.tensor([0, 1, 0], dtype=torch.int32, device="cuda")   # row 1 stores column 0
    v = torch.ones(3, dtype=torch.float32, device="cuda")
    with pytest.raises(hy.HyeigError) as e:
        hy.Matrix(ctx, 2, rp, ci, v, hy.MAT_VALIDATE)
    assert e.value.status == hy.EINVAL


@pytest.mark.parametrize("m", [1, 8, 16])
def test_spmm_block_rows_without_tiles(hy, ctx, m):
    # entries only in rows 0..40 (columns up to 60) and rows 150..199 (their own
    # diagonal block): block rows 2..3 own no tile in either half and must come
    # out zero, every other row as the oracle; Y starts as NaN
    n = 200
    rng = np.random.default_rng(31)
    rows, cols = [], []
    for r in list(range(41)) + list(range(150, 200)):
        hi = 61 if r < 41 else 200
        c = np.unique(rng.integers(r, hi, size=6))
        rows += [r] * c.size
        cols += list(c)
    rows = np.array(rows)
    cols = np.array(cols)
    vals = rng.standard_normal(rows.size).astype(np.float32)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    H = osp.HalfSym(n, rp, cols.astype(np.int32), vals)
    M = hy.matrix_from_csr(ctx, n, rp, cols.astype(np.int32), vals, flags=hy.MAT_VALIDATE)
    for dt, u in ((np.float32, U32), (np.float64, U64)):
        X = sg.normal_block(n, m, 13).astype(dt)
        Yd = torch.full((n, m), float("nan"), dtype=torch.float32 if dt == np.float32 else torch.float64,
                        device="cuda")
        hy.spmm_sym(ctx, M, torch.from_numpy(X).cuda(), Yd)
        Y = Yd.cpu().numpy().astype(np.float64)
        ref = H @ X.astype(np.float64)
        assert np.isfinite(Y).all()
        assert np.all(Y[64:128] == 0.0)
        assert np.all(np.abs(Y - ref) <= _bound(H, X.astype(np.float64), u) + 1e-300)


@pytest.mark.parametrize("n", [1, 5, 31, 33])
@pytest.mark.parametrize("m", [1, 8, 9, 16])
def test_spmm_tiny_orders(hy, ctx, n, m):
    # one partial block row (or one full one and a single row more): every
    # row and column past n must read as absent, in both kernels
    rng = np.random.default_rng(40 + n)
    rows, cols = [], []
    for r in range(n):
        c = np.unique(np.concatenate([[r], rng.integers(r, n, size=4)]))
        rows += [r] * c.size
        cols += list(c)
    rows = np.array(rows)
    cols = np.array(cols, dtype=np.int32)
    vals = rng.standard_normal(rows.size).astype(np.float32)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    H = osp.HalfSym(n, rp, cols, vals)
    M = hy.matrix_from_csr(ctx, n, rp, cols, vals, flags=hy.MAT_VALIDATE)
    for dt, u in ((np.float32, U32), (np.float64, U64)):
        X = sg.normal_block(n, m, 14).astype(dt)
        Yd = torch.full((n, m), float("nan"), dtype=torch.float32 if dt == np.float32 else torch.float64,
                        device="cuda")
        hy.spmm_sym(ctx, M, torch.from_numpy(X).cuda(), Yd)
        Y = Yd.cpu().numpy().astype(np.float64)
        ref = H @ X.astype(np.float64)
        assert np.isfinite(Y).all()
        assert np.all(np.abs(Y - ref) <= _bound(H, X.astype(np.float64), u) + 1e-300)


def test_spmm_argument_errors(hy, ctx, mats):
    spec, H, M = mats["ragged_n1000"]
    X = torch.zeros((spec.n, 40), dtype=torch.float32, device="cuda")
    Y = torch.zeros((spec.n, 40), dtype=torch.float32, device="cuda")
    with pytest.raises(hy.HyeigError) as e:
        hy.spmm_sym(ctx, M, X, Y)   # m = 40 > 32
    assert e.value.status == hy.EINVAL
    Y64 = torch.zeros((spec.n, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(hy.HyeigError) as e:
        hy.spmm_sym(ctx, M, X[:, :8], Y64, acc=hy.F32)
    assert e.value.status == hy.EUNSUPPORTED


@pytest.mark.parametrize("n", [1, 37, 4096 + 3, 200_001])
@pytest.mark.parametrize("ka,kb", [(8, 8), (48, 48), (16, 5), (64, 33)])
def test_gram_modes(hy, ctx, n, ka, kb):
    A = sg.normal_block(n, ka, 1)
    B = sg.normal_block(n, kb, 2)
    ref = A.T @ B
    scale = np.abs(A).T @ np.abs(B)
    G = torch.empty(ka * kb, dtype=torch.float64, device="cuda")
    hy.gram(ctx, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), G, mode=hy.MMA_F64)
    Gh = G.cpu().numpy().reshape(kb, ka).T
    assert np.all(np.abs(Gh - ref) <= _gamma(n, U64) * scale + 1e-300)
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    ref32 = A32.astype(np.float64).T @ B32.astype(np.float64)
    hy.gram(ctx, torch.from_numpy(A32).cuda(), torch.from_numpy(B32).cuda(), G, mode=hy.MMA_F64)
    Gh = G.cpu().numpy().reshape(kb, ka).T
    assert np.all(np.abs(Gh - ref32) <= _gamma(n, U64) * scale + 1e-300)
    hy.gram(ctx, torch.from_numpy(A32).cuda(), torch.from_numpy(B32).cuda(), G, mode=hy.MMA_F32)
    Gh = G.cpu().numpy().reshape(kb, ka).T
    assert np.all(np.abs(Gh - ref32) <= _gamma(n, U32) * scale + 1e-300)
    hy.gram(ctx, torch.from_numpy(A32).cuda(), torch.from_numpy(B32).cuda(), G, mode=hy.MMA_SPLIT_BF16)
    Gh = G.cpu().numpy().reshape(kb, ka).T
    # hi/lo BF16 split keeps ~16 significant bits per factor; the dropped lo*lo
    # term is below 2^-16 relative per product
    assert np.all(np.abs(Gh - ref32) <= (2.0 ** -15 + _gamma(n, U32)) * scale + 1e-300)


def test_gram_without_rows(hy, ctx):
    # n = 0 (valid operand pointers, no rows): G = 0, written by a fill kernel
    X = torch.zeros((10, 8), dtype=torch.float64, device="cuda")
    for ka, kb in ((8, 8), (5, 3)):
        G = torch.full((ka * kb,), float("nan"), dtype=torch.float64, device="cuda")
        st = hy._lib.hyeig_gram(ctx.h, 0, ka, hy._ptr(X), 8, kb, hy._ptr(X), 8, hy.F64, hy.MMA_F64, hy._ptr(G))
        assert st == hy.OK
        assert torch.all(G == 0)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("n,k,m,beta", [(1000, 48, 16, 0.0), (4099, 24, 8, 0.5), (33, 5, 3, -1.0), (70000, 64, 32, 0.0)])
def test_block_update(hy, ctx, dt, n, k, m, beta):
    npdt = np.float32 if dt == "f32" else np.float64
    u = U32 if dt == "f32" else U64
    S = sg.normal_block(n, k, 3).astype(npdt)
    C = sg.normal_block(k, m, 4)
    Y0 = sg.normal_block(n, m, 5).astype(npdt)
    Cd = torch.from_numpy(np.asfortranarray(C).ravel(order="F")).cuda()
    Yd = torch.from_numpy(Y0.copy()).cuda()
    hy.block_update(ctx, torch.from_numpy(S).cuda(), Cd, Yd, beta=beta)
    Cr = C.astype(npdt).astype(np.float64)   # coefficients are used in the data type
    ref = S.astype(np.float64) @ Cr + beta * Y0.astype(np.float64)
    bound = _gamma(k + 2, u) * (np.abs(S.astype(np.float64)) @ np.abs(Cr) + abs(beta) * np.abs(Y0)) + 1e-300
    assert np.all(np.abs(Yd.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_cholqr_identities(hy, ctx, dt):
    npdt = np.float32 if dt == "f32" else np.float64
    n, m = 100_003, 16
    X = sg.normal_block(n, m, 11).astype(npdt)
    Xd = torch.from_numpy(X.copy()).cuda()
    R = torch.empty(m * m, dtype=torch.float64, device="cuda")
    hy.cholqr(ctx, Xd, passes=2, R=R)
    Q = Xd.cpu().numpy().astype(np.float64)
    Rh = R.cpu().numpy().reshape(m, m).T
    u = U32 if dt == "f32" else U64
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) < 50 * m * u * 10
    assert np.allclose(Rh, np.triu(Rh)) and np.all(np.diag(Rh) > 0)
    np.testing.assert_allclose(Q @ Rh, X.astype(np.float64), atol=200 * u * np.abs(X).max())
    # R against the oracle's CholeskyQR of the same data
    Qo, Ro = odense.cholqr(X.astype(np.float64), passes=2)
    np.testing.assert_allclose(Rh, Ro, rtol=0, atol=100 * u * np.abs(Ro).max())


def test_cholqr_rank_deficient(hy, ctx):
    X = sg.normal_block(1000, 4, 1).astype(np.float32)
    X[:, 3] = X[:, 1]
    Xd = torch.from_numpy(X).cuda()
    with pytest.raises(hy.HyeigError) as e:
        hy.cholqr(ctx, Xd, passes=1)
    assert e.value.status == hy.ENOTSPD


def test_queued_copies_many_calls_before_a_sync(hy, ctx):
    # the device form of rayleigh_ritz queues its results through the pinned
    # copy ring without waiting; 40 calls in a row (more than the ring's slots)
    # with distinct pencils, read back only afterwards, must each carry their own
    outs, refs = [], []
    for t in range(40):
        Z = sg.normal_block(24, 24, 100 + t)
        A = Z + Z.T
        Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
        outs.append(hy.rayleigh_ritz(ctx, Ad, None, 6, on_device=True))
        refs.append(np.linalg.eigvalsh(A)[:6])
    torch.cuda.synchronize()
    for (thd, Cd, _), ref in zip(outs, refs):
        np.testing.assert_allclose(thd.cpu().numpy(), ref, rtol=1e-10, atol=1e-10)


def test_rayleigh_ritz_against_oracle(hy, ctx):
    Z = sg.normal_block(48, 48, 1)
    A = Z + Z.T
    Y = sg.normal_block(200, 48, 2)
    B = Y.T @ Y
    th, C, cond = hy.rayleigh_ritz(ctx, A, B, 16)
    tho, Co = odense.rayleigh_ritz(A, B, 16)
    np.testing.assert_allclose(th, tho, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(C.T @ B @ C, np.eye(16), atol=1e-9)
    np.testing.assert_allclose(A @ C, B @ C * th[None, :], atol=1e-8)
    ev = np.linalg.eigvalsh(B)
    assert abs(cond - ev[-1] / ev[0]) < 1e-6 * ev[-1] / ev[0]
    # B = I (tridiagonal and block tridiagonal problems) at a larger size
    Z = sg.normal_block(300, 300, 3)
    A = Z + Z.T
    th, C, _ = hy.rayleigh_ritz(ctx, A, None, 10)
    np.testing.assert_allclose(th, np.linalg.eigvalsh(A)[:10], rtol=1e-10, atol=1e-10)
    # on-device pointers
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()   # symmetric: row- and column-major agree
    thd, Cd, _ = hy.rayleigh_ritz(ctx, Ad, None, 10, on_device=True)
    np.testing.assert_allclose(thd.cpu().numpy(), th, rtol=1e-12)
