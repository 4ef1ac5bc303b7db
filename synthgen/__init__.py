"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds no eigensolver arithmetic: it only draws the half-stored symmetric test
matrices and seeded normal start blocks with a counter-based generator
(Philox4x32-10, Salmon et al., SC'11).  The recipe is in ``synthgen.c``.

The matrix shapes stand in for the nuclear CI Hamiltonians of the paper
(Section 3.1, Table 2: half-stored, 478-636 stored entries per row, low end of
the spectrum wanted); those matrices are not available, so these synthetic
banded 32x32-tile matrices are used instead.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synthgen.c")
_LIB_PATH = os.path.join(_HERE, "libsynthgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libsynthgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32, u32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_double
        vp = ctypes.c_void_p
        lib.sg_philox4x32_10.argtypes = [vp, vp, vp]
        lib.sg_philox4x32_10.restype = None
        lib.sg_gen_rowcounts.argtypes = [i64, i32, i64, dbl, u32, i64, i64, vp]
        lib.sg_gen_rowcounts.restype = i64
        lib.sg_gen_fill.argtypes = [i64, i32, i64, dbl, u32, i64, i64, vp, vp, vp]
        lib.sg_gen_fill.restype = None
        lib.sg_gen_csr.argtypes = [i64, i32, i64, dbl, u32, vp, vp, vp]
        lib.sg_gen_csr.restype = i64
        lib.sg_normal_block_f64.argtypes = [i64, i32, i64, u32, u32, vp]
        lib.sg_normal_block_f64.restype = None
        lib.sg_tile_cols.argtypes = [i64, i32, i64, u32, i64, vp]
        lib.sg_tile_cols.restype = i32
        lib.sg_diag_value.argtypes = [i64, u32, i64]
        lib.sg_diag_value.restype = ctypes.c_float
        _lib = lib
    return _lib


@dataclass(frozen=True)
class MatrixSpec:
    """Generator parameters: order n, upper tiles per block row t, band w (in
    block rows), entry probability p, seed."""
    n: int
    t: int
    w: int
    p: float
    seed: int

    @property
    def nbr(self) -> int:
        return (self.n + 31) // 32


# The three matrix workloads (the stand-ins for the paper's Hamiltonians).
SMALL = MatrixSpec(n=8192, t=15, w=64, p=0.25, seed=100)          # n=8192, 256 block rows
SCALE = MatrixSpec(n=2_097_152, t=24, w=4096, p=0.3, seed=101)    # n=2,097,152
LARGE = MatrixSpec(n=33_554_432, t=48, w=16384, p=0.25, seed=102) # n=33,554,432


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, dtype=np.uint32)
    lib.sg_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def tile_cols(spec: MatrixSpec, i: int) -> np.ndarray:
    lib = _load()
    out = np.zeros(max(spec.t, 1), dtype=np.int32)
    k = lib.sg_tile_cols(spec.nbr, min(spec.t, 1024), spec.w, spec.seed & 0xFFFFFFFF, i, out.ctypes.data)
    return out[:k].copy()


def gen_csr(spec: MatrixSpec):
    """Upper triangle (diagonal included) as CSR: (rowptr int64[n+1],
    colidx int32[nnz], vals float32[nnz]); rows ascending in column, diagonal
    first."""
    lib = _load()
    rowptr = np.zeros(spec.n + 1, dtype=np.int64)
    nnz = lib.sg_gen_csr(spec.n, spec.t, spec.w, spec.p, spec.seed & 0xFFFFFFFF, rowptr.ctypes.data, None, None)
    colidx = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=np.float32)
    lib.sg_gen_fill(spec.n, spec.t, spec.w, spec.p, spec.seed & 0xFFFFFFFF, 0, spec.nbr,
                    rowptr.ctypes.data, colidx.ctypes.data, vals.ctypes.data)
    return rowptr, colidx, vals


def gen_block_rows(spec: MatrixSpec, i0: int, i1: int):
    """CSR of block rows [i0, i1) only: (local rowptr starting at 0, colidx, vals)."""
    lib = _load()
    i1 = min(i1, spec.nbr)
    r0, r1 = 32 * i0, min(32 * i1, spec.n)
    counts = np.zeros(r1 - r0 + 1, dtype=np.int64)
    lib.sg_gen_rowcounts(spec.n, spec.t, spec.w, spec.p, spec.seed & 0xFFFFFFFF, i0, i1, counts[1:].ctypes.data)
    rowptr = np.cumsum(counts)
    nnz = int(rowptr[-1])
    colidx = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=np.float32)
    lib.sg_gen_fill(spec.n, spec.t, spec.w, spec.p, spec.seed & 0xFFFFFFFF, i0, i1,
                    rowptr.ctypes.data, colidx.ctypes.data, vals.ctypes.data)
    return rowptr, colidx, vals


def diag_value(spec: MatrixSpec, k: int) -> float:
    return float(_load().sg_diag_value(spec.n, spec.seed & 0xFFFFFFFF, k))


def normal_block(n: int, m: int, seed: int, stream: int = 4) -> np.ndarray:
    """Seeded N(0,1) block, n x m, row-major float64."""
    lib = _load()
    out = np.empty((n, m), dtype=np.float64)
    lib.sg_normal_block_f64(n, m, m, seed & 0xFFFFFFFF, stream, out.ctypes.data)
    return out


def start_block(spec: MatrixSpec, m: int) -> np.ndarray:
    """Start block X0 for a solve on ``spec``: seeded N(0,1) with seed = matrix seed + 1."""
    return normal_block(spec.n, m, spec.seed + 1, 4)


def expected_nnz(spec: MatrixSpec) -> float:
    """Expected number of stored entries: the diagonal, p times the strict upper
    part of each diagonal tile and p times the entries of each upper tile
    (min(t, band, block rows to the right) tiles per block row), columns past n
    left out."""
    nbr = spec.nbr
    i = np.arange(nbr, dtype=np.int64)
    ntile = np.minimum(np.minimum(spec.t, spec.w), nbr - 1 - i)
    full = ntile.sum() * 1024.0
    # the last block column may be partial: its tiles keep 32 * (n - 32 (nbr - 1)) entries
    tail = spec.n - 32 * (nbr - 1)
    if tail < 32:
        # tiles in the last block column: every block row within the band of it
        # draws it with probability (its tile count) / (its candidate count)
        cand = np.minimum(spec.w, nbr - 1 - i)
        hit = np.where((nbr - 1 - i >= 1) & (nbr - 1 - i <= spec.w), ntile / np.maximum(cand, 1), 0.0)
        full -= hit.sum() * 32 * (32 - tail)
    diag_tiles = (nbr - 1) * 496.0 + tail * (tail - 1) / 2.0
    return spec.n + spec.p * (full + diag_tiles)


def device_csr(spec: MatrixSpec, device: str = "cuda:0", chunk: int = 16384, log=None):
    """The whole upper-triangle CSR generated in chunks of block rows on the
    host and copied into device arrays as it goes, so that the host holds one
    chunk at a time.  Returns (rowptr int64[n+1], colidx int32[cap],
    vals float32[cap], nnz) as torch tensors on ``device``; entries past nnz are
    unused (the arrays are sized from the expected count with a wide margin)."""
    import time
    import torch
    est = expected_nnz(spec)
    cap = int(est + 64.0 * np.sqrt(est) + 1_000_000)
    rowptr = torch.empty(spec.n + 1, dtype=torch.int64, device=device)
    colidx = torch.empty(cap, dtype=torch.int32, device=device)
    vals = torch.empty(cap, dtype=torch.float32, device=device)
    off = 0
    t0 = time.time()
    for i0 in range(0, spec.nbr, chunk):
        i1 = min(spec.nbr, i0 + chunk)
        brp, bci, bv = gen_block_rows(spec, i0, i1)
        cnt = int(brp[-1])
        if off + cnt > cap:
            raise RuntimeError("device_csr: %d entries exceed the reserved %d" % (off + cnt, cap))
        r0, r1 = 32 * i0, min(32 * i1, spec.n)
        rowptr[r0:r1 + 1].copy_(torch.from_numpy(brp + off))
        colidx[off:off + cnt].copy_(torch.from_numpy(bci))
        vals[off:off + cnt].copy_(torch.from_numpy(bv))
        off += cnt
        if log is not None:
            log("device_csr: block rows %d/%d, %d entries, %.1f s" % (i1, spec.nbr, off, time.time() - t0))
    if str(device).startswith("cuda"):
        torch.cuda.synchronize(device)
    return rowptr, colidx, vals, off
