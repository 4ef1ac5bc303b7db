"""Pins for the seeded input generator (not the method): Philox known answers,
an independent pure-Python re-implementation of the matrix recipe, CSR
structure and nnz statistics."""
import math
import os

import numpy as np
import pytest

import synthgen as sg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = sg.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# ---- independent pure-Python re-implementation of the recipe ---------------

def _philox(ctr, key):
    c = list(ctr)
    k0, k1 = key
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
    return c


def _normal(w0, w1, branch):
    u1 = (w0 + 0.5) / 4294967296.0
    u2 = (w1 + 0.5) / 4294967296.0
    rad = math.sqrt(-2.0 * math.log(u1))
    ang = 6.283185307179586 * u2
    return rad * (math.sin(ang) if branch else math.cos(ang))


def _py_csr(n, t, w, p, seed):
    nbr = (n + 31) // 32
    thr = math.floor(p * 4294967296.0)
    rows = [[] for _ in range(n)]
    for i in range(nbr):
        hi = min(i + w, nbr - 1)
        cnt = hi - i
        if cnt <= 0:
            cols = []
        elif cnt <= t:
            cols = [i + 1 + q for q in range(cnt)]
        else:
            sel = []
            for jj in range(cnt - t, cnt):
                o = _philox([i, jj - (cnt - t), 0, 0], [seed, 0])
                r = (o[0] * (jj + 1)) >> 32
                sel.append(jj if r in sel else r)
            cols = sorted(i + 1 + s for s in sel)
        for j in [i] + cols:
            for e in range(1024):
                r, c = divmod(e, 32)
                o = _philox([i, j, e // 4, 0], [seed, 1])
                if o[e % 4] >= thr:
                    continue
                if j == i and c <= r:
                    continue
                row, col = 32 * i + r, 32 * j + c
                if row >= n or col >= n:
                    continue
                ov = _philox([i, j, e // 2, 0], [seed, 2])
                rows[row].append((col, float(np.float32(0.5 * _normal(ov[0], ov[1], e & 1)))))
    for k in range(n):
        o = _philox([k >> 1, 0, 0, 0], [seed, 3])
        dk = float(np.float32(20.0 * k / n + 0.1 * _normal(o[0], o[1], k & 1)))
        rows[k].append((k, dk))
        rows[k].sort()
    return rows


@pytest.mark.parametrize("n,t,w,p,seed", [(200, 3, 4, 0.3, 7), (256, 2, 2, 0.25, 100), (97, 5, 9, 0.5, 3)])
def test_generator_matches_python_reimplementation(n, t, w, p, seed):
    rp, ci, v = sg.gen_csr(sg.MatrixSpec(n, t, w, p, seed))
    rows = _py_csr(n, t, w, p, seed)
    assert rp[-1] == sum(len(r) for r in rows)
    for k in range(n):
        cols = ci[rp[k]:rp[k + 1]]
        vals = v[rp[k]:rp[k + 1]]
        assert list(cols) == [c for c, _ in rows[k]]
        np.testing.assert_array_equal(vals, np.array([x for _, x in rows[k]], dtype=np.float32))


def test_structure_and_statistics():
    spec = sg.SMALL
    rp, ci, v = sg.gen_csr(spec)
    n = spec.n
    assert rp[0] == 0 and np.all(np.diff(rp) >= 1)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(ci >= rows) and np.all(ci < n)
    assert np.all(ci[rp[:-1]] == np.arange(n))            # diagonal first
    d = np.diff(ci.astype(np.int64))
    same_row = np.diff(rows) == 0
    assert np.all(d[same_row] > 0)                          # ascending columns
    # expected stored entries: diagonal + strictly upper diagonal-tile draws + off-diagonal tiles
    nbr = spec.nbr
    tiles = sum(min(spec.t, max(0, min(i + spec.w, nbr - 1) - i)) for i in range(nbr))
    draws = tiles * 1024 + nbr * 496
    mean = n + spec.p * draws
    sd = math.sqrt(draws * spec.p * (1 - spec.p))
    assert abs(rp[-1] - mean) < 5 * sd
    # values: off-diagonal entries ~ 0.5 N(0,1); diagonal ~ 20 k/n + 0.1 N(0,1)
    off = v[ci != rows]
    assert abs(off.mean()) < 5 * 0.5 / math.sqrt(off.size)
    assert abs(off.std() - 0.5) < 0.01
    dres = v[rp[:-1]] - 20.0 * np.arange(n) / n
    assert abs(dres.std() - 0.1) < 0.01


def test_block_rows_agree_with_whole_matrix():
    spec = sg.MatrixSpec(3000, 6, 20, 0.3, 11)
    rp, ci, v = sg.gen_csr(spec)
    lrp, lci, lv = sg.gen_block_rows(spec, 30, 60)
    r0, r1 = 32 * 30, 32 * 60
    np.testing.assert_array_equal(lrp, rp[r0:r1 + 1] - rp[r0])
    np.testing.assert_array_equal(lci, ci[rp[r0]:rp[r1]])
    np.testing.assert_array_equal(lv, v[rp[r0]:rp[r1]])


def test_normal_block_is_seeded_and_standard():
    a = sg.normal_block(4096, 16, 5)
    b = sg.normal_block(4096, 16, 5)
    np.testing.assert_array_equal(a, b)
    assert abs(a.mean()) < 0.01 and abs(a.std() - 1) < 0.01
    o = _philox([3, 2, 0, 0], [5, 4])
    assert a[3, 4] == _normal(o[0], o[1], 0) and a[3, 5] == _normal(o[0], o[1], 1)


def test_chunked_device_build_matches_whole_matrix():
    """The chunked builder (one chunk of block rows at a time, copied into
    preallocated arrays) gives the same CSR as the one-shot generator, and the
    expected entry count it sizes the arrays from is close to the drawn one."""
    torch = pytest.importorskip("torch")
    spec = sg.MatrixSpec(n=4000, t=9, w=20, p=0.25, seed=5)
    rp, ci, v = sg.gen_csr(spec)
    drp, dci, dv, nnz = sg.device_csr(spec, "cpu", chunk=7)
    assert nnz == rp[-1] and dci.numel() >= nnz
    assert np.array_equal(drp.numpy(), rp)
    assert np.array_equal(dci.numpy()[:nnz], ci) and np.array_equal(dv.numpy()[:nnz], v)
    for s in (sg.SMALL, spec):
        e = sg.expected_nnz(s)
        got = sg.gen_csr(s)[0][-1]
        assert abs(got - e) < 6 * math.sqrt(e), (s, got, e)
