"""The allocation-free Gram product (hyeig_gram_noalloc) against the allocating
one (hyeig_gram) and the FP64 oracle, called through the C-ABI: two calls in a
row on one device, the second smaller, in every matrix-core mode.  The partial
sums go to the library's fixed per-device buffer, which keeps the previous
call's contents; each call must still give the full result.  Tolerances are the
summation bound gamma_n sum |a_i b_i| of the accumulation type, as for
hyeig_gram."""
import numpy as np
import pytest

import synthgen as sg
from oracle import sparse as osp

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


def _check(hy, ctx, n, ka, kb, seed):
    A = sg.normal_block(n, ka, seed)
    B = sg.normal_block(n, kb, seed + 1)
    scale = np.abs(A).T @ np.abs(B)
    cases = [(A, B, hy.MMA_F64, U64)]
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    cases += [(A32, B32, hy.MMA_F64, U64), (A32, B32, hy.MMA_F32, U32),
              (A32, B32, hy.MMA_SPLIT_BF16, None)]
    for a, b, mode, u in cases:
        ref = osp.gram(a.astype(np.float64), b.astype(np.float64))
        tol = (2.0 ** -15 + _gamma(n, U32)) * scale if u is None else _gamma(n, u) * scale
        Ad, Bd = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        G0 = torch.full((ka * kb,), float("nan"), dtype=torch.float64, device="cuda")
        G1 = torch.full((ka * kb,), float("nan"), dtype=torch.float64, device="cuda")
        hy.gram(ctx, Ad, Bd, G0, mode=mode)
        hy.gram_noalloc(ctx, Ad, Bd, G1, mode=mode)
        g0 = G0.cpu().numpy().reshape(kb, ka).T
        g1 = G1.cpu().numpy().reshape(kb, ka).T
        assert np.isfinite(g1).all()
        assert np.all(np.abs(g1 - ref) <= tol + 1e-300), (n, ka, kb, mode)
        # both entry points within the bound of the oracle, so within twice it of each other
        assert np.all(np.abs(g1 - g0) <= 2 * tol + 1e-300), (n, ka, kb, mode)


@pytest.mark.parametrize("first,second", [((2_000_000, 64, 64), (5_003, 16, 12)),
                                          ((300_001, 48, 40), (37, 8, 8))])
def test_gram_noalloc_two_calls(hy, ctx, first, second):
    # first call: 64 x 64 FP64 partials cap the workgroups at 128 for the 4 MiB
    # buffer (the allocating form uses up to 512); the second reuses the
    # buffer with fewer, smaller partials
    _check(hy, ctx, *first, seed=11)
    _check(hy, ctx, *second, seed=21)


def test_gram_noalloc_empty_and_errors(hy, ctx):
    # n = 0 (valid operand pointers, no rows): G = 0
    X = torch.zeros((10, 8), dtype=torch.float64, device="cuda")
    G = torch.full((64,), float("nan"), dtype=torch.float64, device="cuda")
    st = hy._lib.hyeig_gram_noalloc(ctx.h, 0, 8, hy._ptr(X), 8, 8, hy._ptr(X), 8, hy.F64, hy.MMA_F64, hy._ptr(G))
    assert st == hy.OK
    assert torch.all(G == 0)
    with pytest.raises(hy.HyeigError) as e:
        hy.gram_noalloc(ctx, X, X, G, mode=hy.MMA_F32)
    assert e.value.status == hy.EUNSUPPORTED
    Xw = torch.zeros((10, 80), dtype=torch.float32, device="cuda")
    with pytest.raises(hy.HyeigError) as e:
        hy.gram_noalloc(ctx, Xw, Xw, G)
    assert e.value.status == hy.EINVAL
