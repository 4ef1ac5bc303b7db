"""GPU solver parity: LOBPCG, block Lanczos, batched RMM-DIIS and the hybrids
through the C-ABI, against the FP64 oracle (step-level, same start state) and
against dense LAPACK eigh (end to end)."""
import os

import numpy as np
import pytest

import synthgen as sg
from oracle import solvers
from oracle import sparse as osp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "small_n8192_seed100_spectrum.txt")


def _golden():
    kv = dict(l.split() for l in open(GOLD) if l.strip() and not l.startswith("#"))
    return np.array([float(kv["lambda%d" % (i + 1)]) for i in range(32)]), float(kv["norm2"])


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
def small(hy, ctx):
    spec = sg.SMALL
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSym(spec.n, rp, ci, v)
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v, flags=hy.MAT_BF16 | hy.MAT_ROWSTATS)
    return spec, H, M


@pytest.fixture(scope="module")
def mid(hy, ctx):
    spec = sg.MatrixSpec(1024, 6, 12, 0.25, 6)
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSym(spec.n, rp, ci, v)
    w = np.linalg.eigvalsh(H.dense())
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v, flags=hy.MAT_BF16)
    return spec, H, M, w


def _x0(spec, nb):
    return torch.from_numpy(sg.start_block(spec, nb).astype(np.float32)).cuda()


@pytest.mark.parametrize("nb", [8, 12, 16])
@pytest.mark.parametrize("prec", ["plain", "f32"])
def test_lobpcg_small_workload_against_eigh(hy, ctx, small, prec, nb):
    """n=8192, block 8, 12 or 16 (16: the blocks of [X W P] stored apart; 12:
    rows of 36, the update's inner dimension not a multiple of 16), 8 pairs,
    shifted Jacobi, residual 1e-6 relative to ||H||_2."""
    spec, H, M = small
    lam, hn = _golden()
    precision = hy.PREC_PLAIN_F64 if prec == "plain" else hy.PREC_F32
    p = hy.params_default(k=8, nb=nb, method=hy.LOBPCG, tol=1e-6, hnorm=hn, maxiter=1000, precision=precision)
    X = _x0(spec, nb)
    ev, rs, rep, st, hist = hy.solve_lowest_k(ctx, M, p, X, hist_cap=2000)
    assert st == hy.OK, (rep.iters_front, rs)
    np.testing.assert_allclose(ev, lam[:8], rtol=1e-8)
    assert np.all(rs <= 1e-6)
    assert rep.orth_err < 1e-4
    # independent check of the returned vectors with the oracle's FP64 product
    th, rh, rt, orth = solvers.final_check(H, X[:, :8].cpu().numpy().astype(np.float64), hn)
    np.testing.assert_allclose(th, ev, rtol=1e-12)
    assert np.all(rh <= 1e-6)
    assert rep.spmm_count >= rep.iters_front + 1


@pytest.mark.parametrize("nb", [8, 16])
def test_precision_form_small_workload(hy, ctx, small, nb):
    """The precision form on the n = 8192 matrix (blocks 8 and 16): BF16 stored
    values in the product and split-BF16 Gram sums until the residual reaches
    1e-4 (100 x the tolerance), then FP32 refinement sweeps; FP64 small problems
    and final check.
    Every eigenvalue within 1e-8 relative of dense eigh (the oracle's spectrum),
    every residual <= 1e-6, and the eigenvectors checked by the oracle's FP64
    product; the refinement sweeps are counted."""
    spec, H, M = small
    lam, hn = _golden()
    p = hy.params_default(k=8, nb=nb, method=hy.LOBPCG, tol=1e-6, hnorm=hn, maxiter=1000,
                          precision=hy.PREC_BF16_SPMM)
    X = _x0(spec, nb)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    print("\nBF16 form, n=8192: %d iterations (%d FP32 refinement), eigenvalue errors %s, residuals %s"
          % (rep.iters_front, rep.iters_refine, np.array2string(np.abs(ev - lam[:8]) / np.abs(lam[:8]), precision=2),
             np.array2string(rs, precision=2)))
    assert st == hy.OK
    assert 0 < rep.iters_refine <= rep.iters_front
    np.testing.assert_allclose(ev, lam[:8], rtol=1e-8)
    assert np.all(rs <= 1e-6)
    th, rh, _, _ = solvers.final_check(H, X[:, :8].cpu().numpy().astype(np.float64), hn)
    np.testing.assert_allclose(th, ev, rtol=1e-12)
    assert np.all(rh <= 1e-6)


@pytest.mark.parametrize("nb", [5, 8, 12, 16])
@pytest.mark.parametrize("iters", [1, 3, 10])
def test_lobpcg_step_parity_plain(hy, ctx, mid, iters, nb):
    """Same start block, same number of iterations: the FP64 GPU path and the
    oracle reach the same Ritz values (block 16: [X W P] stored as three arrays;
    5 and 12: odd row lengths, element-wise loads in the update)."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, nb)
    p = hy.params_default(k=5, nb=nb, method=hy.LOBPCG, tol=1e-14, hnorm=hn, maxiter=iters,
                          precision=hy.PREC_PLAIN_F64)
    X = torch.from_numpy(X0.astype(np.float32)).cuda()
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.ENOCONV and rep.iters_front == iters
    # the start block is rounded to FP32 on the GPU side: compare with the oracle
    # started from the same FP32 numbers
    ref = solvers.lobpcg(H, X0.astype(np.float32).astype(np.float64), 5, tol=1e-14, maxiter=iters, hnorm=hn, d=H.d)
    # returned vectors are FP32: the Rayleigh quotient of x + dx moves by about
    # 2 dx^T r, |dx| <= u32 |x|, r the residual of the (unconverged) iterate
    bound = 4 * 2.0 ** -24 * rs * hn + 1e-12 * np.abs(ev)
    assert np.all(np.abs(ev - np.sort(ref.theta[:5])) <= bound)


def test_lobpcg_f32_close_to_plain(hy, ctx, mid):
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, 8).astype(np.float32)
    out = {}
    for name, prec in [("plain", hy.PREC_PLAIN_F64), ("f32", hy.PREC_F32), ("bf16", hy.PREC_BF16_SPMM)]:
        p = hy.params_default(k=5, nb=8, method=hy.LOBPCG, tol=1e-6, hnorm=hn, maxiter=2000, precision=prec)
        X = torch.from_numpy(X0.copy()).cuda()
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
        assert st == hy.OK, name
        out[name] = ev
        np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
        assert np.all(rs <= 1e-6)


def test_block_lanczos_against_eigh_and_oracle(hy, ctx, mid):
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, 8).astype(np.float32)
    p = hy.params_default(k=5, nb=8, method=hy.BLANCZOS, tol=1e-6, hnorm=hn, maxiter=120,
                          precision=hy.PREC_PLAIN_F64)
    X = torch.from_numpy(X0.copy()).cuda()
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.OK
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    ref = solvers.block_lanczos(H, X0.astype(np.float64), 5, tol=0.9e-6, maxiter=120, hnorm=hn)
    assert abs(rep.iters_front - ref.iters) <= 1


def test_single_vector_lanczos(hy, ctx, mid):
    """Block size 1 (the Lanczos method of Section 2.1) for 5 pairs: the start
    vector in the first column of a 5-column X, eigenvalues against dense eigh,
    iteration count (= SpMV count) against the oracle's."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, 1).astype(np.float32)
    X = torch.zeros((spec.n, 5), dtype=torch.float32, device="cuda")
    X[:, :1] = torch.from_numpy(X0).cuda()
    p = hy.params_default(k=5, nb=1, method=hy.BLANCZOS, tol=1e-6, hnorm=hn, maxiter=400,
                          precision=hy.PREC_PLAIN_F64)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.OK, (rep.iters_front, rs)
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    assert np.all(rs <= 1e-6)
    # one vector per product, plus the final check's product of the 5 vectors
    assert rep.spmm_count - 1 == rep.spmv_count - 5 == rep.iters_front
    ref = solvers.block_lanczos(H, X0.astype(np.float64), 5, tol=0.9e-6, maxiter=400, hnorm=hn)
    assert abs(rep.iters_front - ref.iters) <= 1, (rep.iters_front, ref.iters)
    th, rh, _, _ = solvers.final_check(H, X.cpu().numpy().astype(np.float64), hn)
    np.testing.assert_allclose(th, ev, rtol=1e-12)
    # k above the block size is for block Lanczos alone
    with pytest.raises(hy.HyeigError) as e:
        hy.solve_lowest_k(ctx, M, hy.params_default(k=5, nb=1, method=hy.LOBPCG, hnorm=hn), X)
    assert e.value.status == hy.EINVAL


def test_block_lanczos_step_parity(hy, ctx, mid):
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.start_block(spec, 8).astype(np.float32).astype(np.float64)
    for iters in [2, 6]:
        ref = solvers.block_lanczos(H, X0, 5, tol=1e-15, maxiter=iters, hnorm=hn)
        p = hy.params_default(k=5, nb=8, method=hy.BLANCZOS, tol=1e-15, hnorm=hn, maxiter=iters,
                              precision=hy.PREC_PLAIN_F64)
        X = torch.from_numpy(X0.astype(np.float32)).cuda()
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
        assert rep.iters_front == iters
        bound = 4 * 2.0 ** -24 * rs * hn + 1e-12 * np.abs(ev)
        assert np.all(np.abs(ev - ref.theta) <= bound)


def test_rmm_diis_step_parity(hy, ctx, mid):
    """Batched RMM-DIIS sweeps from the same vectors, against the oracle's
    sweeps (FP32 vectors on the GPU)."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    lam, V = np.linalg.eigh(H.dense())
    N = sg.normal_block(spec.n, 4, 3)
    N -= V[:, :4] @ (V[:, :4].T @ N)
    X0 = (V[:, :4] + 1e-2 * N).astype(np.float32)
    st = hy.RmmState(ctx, M, torch.from_numpy(X0).cuda(), s_max=6, tol=1e-14, hnorm=hn)
    th0, rs0, _ = st.get()
    ref0 = solvers.rmm_diis(H, X0.astype(np.float64), k=4, s_max=6, tol=1e-14, maxiter=0, hnorm=hn)
    np.testing.assert_allclose(th0, ref0.theta, rtol=1e-7)
    done = 0
    for sweeps in [1, 2, 3, 5, 8]:
        while done < sweeps:
            st.step()
            done += 1
        ref = solvers.rmm_diis(H, X0.astype(np.float64), k=4, s_max=6, tol=1e-14, maxiter=sweeps, hnorm=hn)
        th, rs, cv = st.get()
        np.testing.assert_allclose(th, ref.theta, rtol=1e-6, atol=1e-6 * hn)
        np.testing.assert_allclose(rs, ref.resid, rtol=0.05, atol=1e-6)


@pytest.mark.parametrize("method", ["lobpcg_rmm", "blanczos_rmm"])
def test_hybrid_against_eigh(hy, ctx, mid, method):
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    m = hy.LOBPCG_RMMDIIS if method == "lobpcg_rmm" else hy.BLANCZOS_RMMDIIS
    p = hy.params_default(k=5, nb=8, method=m, tol=1e-6, hnorm=hn, maxiter=400, switch_rule=hy.SWITCH_TAU,
                          switch_thr=1e-7, precision=hy.PREC_F32)
    X = _x0(spec, 8)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.OK
    assert rep.switched == 1
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    assert np.all(rs <= 1e-6)


@pytest.mark.parametrize("method", ["lobpcg_rmm", "blanczos_rmm"])
def test_hybrid_hands_over_at_front_end_limit(hy, ctx, mid, method):
    """A switch threshold that cannot fire: the front end hands over at its
    iteration limit (a fixed switch point), and after RMM-DIIS a LOBPCG finishes
    if needed (for block Lanczos with nb_back = 12 columns: the refined vectors
    and the next Ritz vectors of the front end)."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    m = hy.LOBPCG_RMMDIIS if method == "lobpcg_rmm" else hy.BLANCZOS_RMMDIIS
    p = hy.params_default(k=5, nb=8, method=m, tol=1e-6, hnorm=hn, maxiter=6, switch_rule=hy.SWITCH_TAU,
                          switch_thr=1e-300, s_max=6, rmm_maxiter=300, maxiter_back=600,
                          nb_back=12 if method == "blanczos_rmm" else 0, precision=hy.PREC_F32)
    X = _x0(spec, 8)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert rep.switched == 1 and rep.iters_front == 6
    assert st == hy.OK, (rep.iters_rmm, rep.iters_back, rs)
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    assert np.all(rs <= 1e-6)
    th, rh, _, _ = solvers.final_check(H, X[:, :5].cpu().numpy().astype(np.float64), hn)
    np.testing.assert_allclose(th, ev, rtol=1e-12)
    assert np.all(rh <= 1e-6)


def test_rmm_diis_coupled_and_decoupled_products(hy, ctx, small):
    """Section 4.2's two ways of running the batched RMM-DIIS once some columns
    have converged: one product over all columns with the converged ones
    frozen (coupled), or one SpMV per unconverged column after c have
    converged (decoupled).  The iterates are the same; the SpMV counts differ."""
    spec, H, M = small
    lam, hn = _golden()
    out = {}
    for c in (0, 1, 3):
        p = hy.params_default(k=5, nb=8, method=hy.BLANCZOS_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=200,
                              switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, s_max=10, rmm_maxiter=300,
                              rmm_decouple=c, precision=hy.PREC_F32)
        X = _x0(spec, 8)
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
        out[c] = (ev, rs, rep, st)
        print("\nRMM-DIIS %s: front %d, sweeps %d, back %d, products %d, SpMVs %d, fallback %d" % (
            "coupled" if c == 0 else "decoupled after %d" % c, rep.iters_front, rep.iters_rmm, rep.iters_back,
            rep.spmm_count, rep.spmv_count, rep.fallback_used))
        assert st == hy.OK and rep.switched == 1
        np.testing.assert_allclose(ev, lam[:5], rtol=1e-8)
        assert np.all(rs <= 1e-6)
    ev0, _, rep0, _ = out[0]
    for c in (1, 3):
        ev, _, rep, _ = out[c]
        assert rep.iters_front == rep0.iters_front and rep.iters_rmm == rep0.iters_rmm
        assert rep.iters_back == rep0.iters_back and rep.fallback_used == rep0.fallback_used
        np.testing.assert_allclose(ev, ev0, rtol=1e-12)
        assert rep.spmv_count <= rep0.spmv_count


@pytest.mark.parametrize("case", ["theta_norm", "no_lock", "stable_basis_plain", "rmm_precond", "refresh_5",
                                  "jacobi_floor", "no_fallback"])
def test_solver_options(hy, ctx, mid, case):
    """Each solver option on the n = 1024 matrix (5 pairs, block 8): the pairs
    against dense eigh, residuals in the chosen normalisation, and the returned
    vectors checked by the oracle's FP64 product."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    kw = dict(k=5, nb=8, method=hy.LOBPCG, tol=1e-6, hnorm=hn, maxiter=2000, precision=hy.PREC_F32)
    if case == "theta_norm":
        kw.update(tol_norm=hy.NORM_THETA)
    elif case == "no_lock":
        kw.update(lock=0)
    elif case == "stable_basis_plain":
        kw.update(basis=1, precision=hy.PREC_PLAIN_F64)
    elif case == "rmm_precond":
        kw.update(method=hy.LOBPCG_RMMDIIS, switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, rmm_precond=1)
    elif case == "refresh_5":
        kw.update(refresh_every=5)
    elif case == "jacobi_floor":
        kw.update(jacobi_floor=0.5)
    elif case == "no_fallback":
        kw.update(method=hy.LOBPCG_RMMDIIS, switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, fallback=0, rmm_maxiter=100)
    p = hy.params_default(**kw)
    X = _x0(spec, 8)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    if case == "no_fallback":
        # RMM-DIIS alone after the switch: converged, or stopped at its sweep limit without LOBPCG
        assert rep.switched == 1 and rep.fallback_used == 0 and rep.iters_back == 0
        if st != hy.OK:
            assert st == hy.ENOCONV and rep.iters_rmm <= 100
            return
    assert st == hy.OK, (case, rep.iters_front, rs)
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    th, rh, rt, _ = solvers.final_check(H, X[:, :5].cpu().numpy().astype(np.float64), hn)
    np.testing.assert_allclose(th, ev, rtol=1e-12)
    if case == "theta_norm":
        assert rep.resid_theta_max <= 1e-6 and np.all(rt <= 1e-6 * 1.001)
    else:
        assert np.all(rs <= 1e-6) and np.all(rh <= 1e-6 * 1.001)


def test_warm_start_from_principal_submatrix(hy, ctx, small):
    """The analogue of the paper's smaller-model-space start vectors: the lowest
    eigenvectors of the leading quarter of H (solved to 1e-3), padded with zeros,
    start LOBPCG on the n = 8192 matrix; it reaches the dense-eigh pairs in
    fewer iterations than the seeded random start."""
    from paper_2305_15552_amd import warmstart as ws
    spec, H, M = small
    lam, hn = _golden()
    rp, ci, v = sg.gen_csr(spec)
    ns = spec.n // 4
    Ms = hy.matrix_from_csr(ctx, ns, *ws.principal_csr(rp, ci, v, ns))
    X0 = _x0(spec, 8)
    Xs = X0[:ns].clone()
    _, _, reps, sts, _ = hy.solve_lowest_k(ctx, Ms, hy.params_default(k=8, nb=8, method=hy.LOBPCG, tol=1e-3,
                                                                       hnorm=hn, maxiter=1000), Xs)
    assert sts == hy.OK
    Xw = torch.zeros_like(X0)
    Xw[:ns] = Xs
    out = {}
    for name, X in (("random", X0.clone()), ("warm", Xw)):
        p = hy.params_default(k=8, nb=8, method=hy.LOBPCG, tol=1e-6, hnorm=hn, maxiter=1000)
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
        assert st == hy.OK
        np.testing.assert_allclose(ev, lam[:8], rtol=1e-8)
        assert np.all(rs <= 1e-6)
        out[name] = rep.iters_front
    print("\nwarm start: %d iterations on the n/4 submatrix, then %d on the full matrix (random start %d)"
          % (reps.iters_front, out["warm"], out["random"]))
    assert out["warm"] < out["random"]
    Ms.close()


@pytest.mark.parametrize("nb", [8, 16])
@pytest.mark.parametrize("prec", ["plain", "f32", "bf16"])
@pytest.mark.parametrize("method", ["lobpcg", "blanczos", "lobpcg_rmm", "blanczos_rmm", "chebfsi", "chebfsi_rmm"])
def test_method_precision_block_grid(hy, ctx, mid, method, prec, nb):
    """Every method in every precision form at blocks 8 and 16 on the n = 1024
    matrix (5 pairs): the dense-eigh pairs at residual 1e-6, or EUNSUPPORTED
    for the BF16 form outside LOBPCG (its FP32 refinement lives there)."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    m = {"lobpcg": hy.LOBPCG, "blanczos": hy.BLANCZOS, "lobpcg_rmm": hy.LOBPCG_RMMDIIS,
         "blanczos_rmm": hy.BLANCZOS_RMMDIIS, "chebfsi": hy.CHEBFSI, "chebfsi_rmm": hy.CHEBFSI_RMMDIIS}[method]
    pr = {"plain": hy.PREC_PLAIN_F64, "f32": hy.PREC_F32, "bf16": hy.PREC_BF16_SPMM}[prec]
    p = hy.params_default(k=5, nb=nb, method=m, tol=1e-6, hnorm=hn, maxiter=600, switch_rule=hy.SWITCH_TAU,
                          switch_thr=1e-7, s_max=10, rmm_maxiter=300, precision=pr)
    X = _x0(spec, nb)
    if prec == "bf16" and method not in ("lobpcg", "lobpcg_rmm"):
        with pytest.raises(hy.HyeigError) as e:
            hy.solve_lowest_k(ctx, M, p, X)
        assert e.value.status == hy.EUNSUPPORTED
        return
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.OK, (method, prec, nb, rep.iters_front, rep.iters_rmm, rep.iters_back, rs)
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    assert np.all(rs <= 1e-6)
    assert rep.orth_err < 1e-4


def test_hybrid_resid_switch_small(hy, ctx, small):
    spec, H, M = small
    lam, hn = _golden()
    p = hy.params_default(k=8, nb=8, method=hy.LOBPCG_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=1000,
                          switch_rule=hy.SWITCH_RESID, switch_thr=1e-4, precision=hy.PREC_F32)
    X = _x0(spec, 8)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.OK and rep.switched == 1
    np.testing.assert_allclose(ev, lam[:8], rtol=1e-8)


def test_norm_estimate(hy, ctx, small):
    spec, H, M = small
    lam, hn = _golden()
    p = hy.params_default(k=4, nb=8, method=hy.LOBPCG, tol=1e-6, hnorm=0.0, maxiter=2000)
    X = _x0(spec, 8)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert 0.9 * hn <= rep.hnorm_used <= hn * (1 + 1e-9)
    np.testing.assert_allclose(ev, lam[:4], rtol=1e-8)


def test_solver_errors(hy, ctx, small):
    spec, H, M = small
    X = _x0(spec, 8)
    with pytest.raises(hy.HyeigError) as e:
        hy.solve_lowest_k(ctx, M, hy.params_default(k=9, nb=8), X)
    assert e.value.status == hy.EINVAL
    # the BF16 form has its FP32 refinement in LOBPCG only
    with pytest.raises(hy.HyeigError) as e:
        hy.solve_lowest_k(ctx, M, hy.params_default(k=8, nb=8, method=hy.BLANCZOS, hnorm=35.0,
                                                    precision=hy.PREC_BF16_SPMM), X)
    assert e.value.status == hy.EUNSUPPORTED
    # guard block of the LOBPCG after block Lanczos outside k..32
    for nbb in (7, 33):
        with pytest.raises(hy.HyeigError) as e:
            hy.solve_lowest_k(ctx, M, hy.params_default(k=8, nb=8, method=hy.BLANCZOS_RMMDIIS, nb_back=nbb), X)
        assert e.value.status == hy.EINVAL
    # iteration limit: ENOCONV with the best results so far filled in
    p = hy.params_default(k=8, nb=8, maxiter=2, hnorm=35.0)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.ENOCONV and np.all(np.isfinite(ev)) and rep.iters_front == 2
    # a start block with a NaN
    Xn = _x0(spec, 8)
    Xn[5, 3] = float("nan")
    with pytest.raises(hy.HyeigError) as e:
        hy.solve_lowest_k(ctx, M, hy.params_default(k=8, nb=8, hnorm=35.0), Xn)
    assert e.value.status in (hy.ENUMERIC, hy.ENOTSPD)


@pytest.mark.parametrize("k", [5, 8])
def test_hybrid_phases_match_oracle(hy, ctx, small, k):
    """LOBPCG (block 8) -> RMM-DIIS (tau < 1e-7) on the n=8192 matrix in the
    plain FP64 form, against the FP64 oracle's hybrid with the same rules: the
    front-end iterations, the RMM-DIIS sweeps until the stagnation guard hands
    the block back, and the LOBPCG iterations after the hand-back (resumed from
    the front end's state with X merged with the refined vectors) each match
    within one.  The library aims at 0.9 tol
    internally, so the oracle runs at that tolerance.  Eigenvalues within 1e-8
    of dense eigh."""
    spec, H, M = small
    lam, hn = _golden()
    p = hy.params_default(k=k, nb=8, method=hy.LOBPCG_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=1000,
                          switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, s_max=10, rmm_maxiter=300,
                          precision=hy.PREC_PLAIN_F64, precond=hy.PRECOND_JACOBI)
    X = _x0(spec, 8)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
    assert st == hy.OK, (rep.iters_front, rep.iters_rmm, rep.iters_back, rs)
    X0 = sg.start_block(spec, 8).astype(np.float32).astype(np.float64)
    fr, rm, back = solvers.hybrid(H, X0, k, front="lobpcg", switch="tau", switch_thr=1e-7, tol=0.9e-6, hnorm=hn,
                                  d=H.d, s_max=10, rmm_maxiter=300, max_front=1000)
    oracle = (fr.iters, rm.iters if rm else 0, back.iters if back else 0)
    gpu = (rep.iters_front, rep.iters_rmm, rep.iters_back)
    print("\nk=%d phases front/RMM-DIIS/back: GPU %s, oracle %s" % (k, gpu, oracle))
    assert all(abs(a - b) <= 1 for a, b in zip(gpu, oracle)), (gpu, oracle)
    assert (rep.fallback_used == 1) == (back is not None)
    # the hand-back resumed with X merged with the refined vectors, on both sides
    if back is not None:
        assert back.events[0][1] == "merged" and rep.merged_back == 1
    np.testing.assert_allclose(ev, lam[:k], rtol=1e-8)


def test_rmm_diis_collapsed_columns_are_not_a_result(hy, ctx, mid):
    """An early fixed switch (2 LOBPCG iterations, 5 pairs, block 8) on the
    n=1024 matrix in the plain FP64 form.  Without the stagnation guard and
    hand-back, RMM-DIIS drives columns onto the same eigenpair: every column's
    residual is below the tolerance, but wanted pairs are missing.  The solve
    must not report success: status ENOCONV, with the orthogonality error of
    the returned block showing the collapse (the oracle's hybrid flags the same
    block).  With the guard and hand-back it returns the dense eigh pairs."""
    spec, H, M, w = mid
    hn = float(np.max(np.abs(w)))
    X0 = sg.normal_block(spec.n, 8, 101).astype(np.float32)
    p = hy.params_default(k=5, nb=8, method=hy.LOBPCG_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=1000,
                          switch_rule=hy.SWITCH_ITERS, switch_thr=2, s_max=10, rmm_maxiter=300, fallback=0,
                          precision=hy.PREC_PLAIN_F64, precond=hy.PRECOND_JACOBI)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, torch.from_numpy(X0).cuda())
    print("\nno hand-back: status %d, RMM-DIIS sweeps %d, orthogonality error %.2e, max residual %.2e"
          % (st, rep.iters_rmm, rep.orth_err, rs.max()))
    assert st == hy.ENOCONV
    assert rep.orth_err > 0.5 and rep.events_stagnation >= 1
    fr, rm, back = solvers.hybrid(H, X0.astype(np.float64), 5, front="lobpcg", switch="iters", switch_thr=2,
                                  tol=0.9e-6, hnorm=hn, d=H.d, fallback=False, rmm_maxiter=300)
    assert rm.events[-1][1] == "collapse" and abs(rm.iters - rep.iters_rmm) <= 1, (rm.iters, rep.iters_rmm)
    p = hy.params_default(k=5, nb=8, method=hy.LOBPCG_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=1000,
                          switch_rule=hy.SWITCH_ITERS, switch_thr=2, s_max=10, rmm_maxiter=300, fallback=1,
                          precision=hy.PREC_PLAIN_F64, precond=hy.PRECOND_JACOBI)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, torch.from_numpy(X0).cuda())
    assert st == hy.OK and rep.fallback_used == 1
    np.testing.assert_allclose(ev, w[:5], rtol=1e-8)
    assert rep.orth_err < 1e-6


@pytest.mark.parametrize("prec", ["plain", "f32"])
def test_report_splits_matrix_core_products(hy, ctx, small, prec):
    """The report's matrix-core share of the products (hyeig_report.spmm_mc_*):
    with block 16 every LOBPCG product of W has 9-16 columns until columns lock,
    so most products run on the matrix cores; their count, time and bytes are a
    part of all products', and the bytes are the per-launch algorithmic formula
    nnz (4 + 4) + 8 (n + 1) + n m (s_x + s_y) summed over those launches."""
    spec, H, M = small
    p = hy.params_default(k=8, nb=16, method=hy.LOBPCG, tol=1e-6, hnorm=0.0, maxiter=500,
                          precision=hy.PREC_PLAIN_F64 if prec == "plain" else hy.PREC_F32,
                          precond=hy.PRECOND_JACOBI)
    ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, _x0(spec, 16))
    assert st == hy.OK
    assert 0 < rep.spmm_mc_count < rep.spmm_count
    assert 0.0 < rep.ms_spmm_mc < rep.ms_spmm
    assert 0.0 < rep.bytes_spmm_mc < rep.bytes_spmm
    nnz = H.U.nnz
    es = 8 if prec == "plain" else 4
    lo = nnz * 8 + 8 * (spec.n + 1) + spec.n * 9 * 2 * es
    hi = nnz * 8 + 8 * (spec.n + 1) + spec.n * 16 * 2 * es
    assert lo * rep.spmm_mc_count <= rep.bytes_spmm_mc <= hi * rep.spmm_mc_count
