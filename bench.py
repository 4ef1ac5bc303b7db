"""Benchmark: time to the k lowest eigenpairs at relative residual 1e-6 on one
MI355X, with the SpMM's achieved HBM bandwidth, the plain FP64 form (the
headline, the paper's arithmetic) and the chosen mixed-precision form beside it.

Workload (one step = one full solve of the hot path on resident inputs):
  synthetic half-stored symmetric matrix, n = 2,097,152 (65,536 block rows of
  32x32 tiles), 24 upper tiles per block row in (i, i+4096], entry probability
  0.3, seed 101; hybrid LOBPCG (block 16) -> RMM-DIIS on the 10 lowest pairs,
  switching when the largest relative residual falls below 1e-3; shifted
  Jacobi preconditioner; relative residual ||Hx - theta x|| / ||H||_2 <= 1e-6.
Plain form (value, roofline): FP64 blocks and FP64 accumulation in every
product, FP32 stored values (the matrix itself).  Chosen form (chosen_f32):
FP32 blocks, FP32 sums in the products, FP64 small problems and Gram sums,
FP64-accumulated final check.  Eigenvalues are compared with the FP64
oracle's reference spectrum of this matrix (tests/golden).

    python bench.py [--gpus 1] [--steps 10] [--warmup 1]

The large single-GPU instance (n = 33,554,432, block Lanczos -> RMM-DIIS, 8
pairs) runs with --workload large (use --steps 1 --warmup 0: one solve takes
about a minute, the matrix about a minute of host generation).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to k eigenpairs @resid 1e-6; SpMM HBM GB/s %peak; plain vs chosen form"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def golden_scale():
    """The oracle's reference for the n=2,097,152 matrix (tests/golden, written
    by make_c2_spectrum.py through oracle/ only), or None."""
    path = os.path.join(ROOT, "tests", "golden", "scale_n2097152_seed101_spectrum.txt")
    if not os.path.exists(path):
        return None
    kv = dict(l.split() for l in open(path) if l.strip() and not l.startswith("#"))
    return kv


def cpu_baseline(spec, nb, k, hnorm, sample_iters=3):
    """The FP64 oracle as it stands, timed on this host on a bounded sample of
    the workload: the whole n=2,097,152 matrix in the oracle's threaded product
    (oracle.sparse.HalfSymOMP, plain C with OpenMP on every host thread) and
    ``sample_iters`` iterations of oracle.solvers.lobpcg (block 16, 10 pairs,
    shifted diagonal, FP64) from the benchmark's start block.  The time per
    iteration (its product and its dense work through numpy/BLAS) is scaled by
    the oracle's own iteration count to relative residual 1e-6 on this matrix,
    from its reference run (tests/golden/make_c2_spectrum.py, plain LOBPCG);
    the set-up (orthonormalisation, first product and Rayleigh-Ritz) is added
    once."""
    import numpy as np
    import synthgen as sg
    from oracle import sparse as osp
    from oracle import solvers as osolv
    gold = golden_scale()
    t_start = time.time()
    rp, ci, v = sg.gen_csr(spec)
    H = osp.HalfSymOMP(spec.n, rp, ci, v)
    del rp, ci, v
    threads = H.nthreads()
    stamps = []

    def stop(it, theta, rel):
        stamps.append(time.time())
        return False

    t0 = time.time()
    osolv.lobpcg(H, sg.start_block(spec, nb), k, tol=1e-6, maxiter=sample_iters, hnorm=hnorm, d=H.d, stop=stop)
    t_setup = stamps[0] - t0
    per_iter = float(np.median(np.diff(stamps)))
    iters = int(gold["oracle_iters_to_1e-6"]) if gold else None
    est = t_setup + iters * per_iter if iters else None
    del H
    # a whole oracle solve where one fits in seconds: LOBPCG (block 8, 8 pairs,
    # shifted Jacobi, 1e-6) on the n = 8192 matrix, scipy product
    sm = sg.SMALL
    srp, sci, sv = sg.gen_csr(sm)
    Hs = osp.HalfSym(sm.n, srp, sci, sv)
    gsm = os.path.join(ROOT, "tests", "golden", "small_n8192_seed100_spectrum.txt")
    kv = dict(l.split() for l in open(gsm) if l.strip() and not l.startswith("#"))
    t0 = time.time()
    rs = osolv.lobpcg(Hs, sg.start_block(sm, 8), 8, tol=1e-6, maxiter=1000, hnorm=float(kv["norm2"]), d=Hs.d)
    small = {"workload": "n=8192 (seed 100) LOBPCG block 8, 8 lowest pairs, tol 1e-6, shifted Jacobi, FP64 oracle "
                         "(products by scipy on one thread, dense work by numpy/BLAS on every host thread)",
             "time_s": round(time.time() - t0, 3), "iterations": rs.iters, "converged": bool(rs.converged)}
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        threadpool_limits = None
    if threadpool_limits is not None:
        # the same solve with BLAS held to one thread: the oracle on one core
        t0 = time.time()
        with threadpool_limits(limits=1):
            osolv.lobpcg(Hs, sg.start_block(sm, 8), 8, tol=1e-6, maxiter=1000, hnorm=float(kv["norm2"]), d=Hs.d)
        small["time_s_one_core"] = round(time.time() - t0, 3)
    try:
        ram_gb = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES") / 1e9
    except (ValueError, OSError):
        ram_gb = None
    return {
        "value": round(est, 1) if est else None, "unit": "s", "cores": threads, "kind": "oracle",
        "nproc": os.cpu_count(), "host_ram_GB": round(ram_gb, 1) if ram_gb else None,
        "per_iteration_s": round(per_iter, 3), "setup_s": round(t_setup, 3),
        "oracle_iters_to_1e-6": iters, "small_full_solve": small,
        "sample": ("FP64 oracle on this host: %d LOBPCG iterations (block %d, %d pairs, shifted diagonal) of "
                   "oracle.solvers.lobpcg on the whole n=%d matrix, products by oracle.sparse.HalfSymOMP on %d "
                   "OpenMP threads, dense work by numpy/BLAS; %.2f s per iteration (median), %.2f s set-up; "
                   "scaled by the oracle's own %s iterations to relative residual 1e-6 on this matrix (its "
                   "reference run, plain LOBPCG, tests/golden/make_c2_spectrum.py); sample took %.1f s"
                   % (sample_iters, nb, k, spec.n, threads, per_iter, t_setup, iters, time.time() - t_start)),
    }


def counted_traffic(name="spmm_mma64_c2_m16_hbm_counters.txt"):
    """HBM bytes per product launch from a committed rocprofv3 counter summary,
    or None when the product kernel's source has changed since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2305_15552_amd", "csrc", "spmm.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if ("sha256 " + sha) not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return float(line.split(":")[1])
    return None


def spmm_bytes(nnz, n, m, sv, sx, sy):
    """Algorithmic bytes of one product: the upper triangle read once as CSR
    (values + 4-byte column index), the row pointer, X read and Y written."""
    return nnz * (sv + 4) + 8 * (n + 1) + n * m * (sx + sy)


def product_table(ctx, M, spec, nnz, forms, reps=20, warm=5):
    """The product alone at several widths (HIP events, median and IQR of
    ``reps`` launches after ``warm`` untimed ones): time, algorithmic GB/s and GFLOP/s, and the
    SpMM/SpMV throughput ratio the paper uses for its effective SpMV count
    (Section 4.2, Tables 12-13: GFLOP/s at width m over GFLOP/s at width 1)."""
    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy
    out = []
    for m, xdt, ydt in forms:
        X = torch.from_numpy(sg.normal_block(spec.n, m, 7)).to(xdt).cuda()
        Y = torch.empty((spec.n, m), dtype=ydt, device="cuda")
        for _ in range(warm):
            hy.spmm_sym(ctx, M, X, Y)
        ts = []
        for _ in range(reps):
            hy.spmm_sym(ctx, M, X, Y)
            ts.append(ctx.last_spmm_ms())
        ms = float(np.median(ts))
        q1, q3 = np.percentile(ts, [25, 75])
        b = spmm_bytes(nnz, spec.n, m, 4, 8 if xdt == torch.float64 else 4, 8 if ydt == torch.float64 else 4)
        gf = 2.0 * m * (2.0 * nnz - spec.n) / ms / 1e6
        out.append({"m": m, "x": "f64" if xdt == torch.float64 else "f32",
                    "accumulate": "f64" if ydt == torch.float64 else "f32", "median_ms": round(ms, 3),
                    "iqr_ms": round(float(q3 - q1), 4), "launches": reps,
                    "algorithmic_GBps": round(b / ms / 1e6, 1), "frac": round(b / ms / 1e6 / HBM_PEAK_GBS, 4),
                    "GFLOPs": round(gf, 1)})
        log("bench: product m=%d x %s acc %s: %.3f ms, %.0f GB/s, %.0f GFLOP/s"
            % (m, out[-1]["x"], out[-1]["accumulate"], ms, b / ms / 1e6, gf))
        del X, Y
    # SpMM/SpMV throughput ratio within each form (the same x and accumulation types)
    for r in out:
        base = [q for q in out if q["m"] == 1 and q["x"] == r["x"] and q["accumulate"] == r["accumulate"]]
        if base:
            r["spmm_spmv_ratio"] = round(r["GFLOPs"] / base[0]["GFLOPs"], 2)
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(nbytes=1 << 31, reps=5):
    """Device-to-device copy rate (read + write bytes per second) of a buffer
    far larger than the caches: the practical streaming ceiling beside the
    8 TB/s peak."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / s / 1e9


def spmm_only(spec, m, args):  # noqa: C901
    """The product alone at the benchmark's size, plus a device copy of a known
    number of bytes (the calibration for HBM byte counters)."""
    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy
    rp, ci, v = sg.gen_csr(spec)
    nnz = int(rp[-1])
    ctx = hy.Context(0)
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v)
    del rp, ci, v
    f64 = args.spmm_dtype == "f64"
    X = torch.from_numpy(sg.normal_block(spec.n, m, 7)).to(torch.float64 if f64 else torch.float32).cuda()
    Y = torch.empty_like(X)
    for _ in range(args.warmup):
        hy.spmm_sym(ctx, M, X, Y)
    ts = []
    for _ in range(args.steps):
        hy.spmm_sym(ctx, M, X, Y)
        ts.append(ctx.last_spmm_ms())
    C = torch.empty_like(X)
    torch.cuda.synchronize()
    C.copy_(X)  # reads and writes n * m * element-size bytes
    torch.cuda.synchronize()
    ms = float(np.median(ts))
    es = 8 if f64 else 4
    b = spmm_bytes(nnz, spec.n, m, 4, es, es)
    kern = ("k_spmm_sym_mma2<%s>" % ("double, double" if f64 else "float, float")) if 9 <= m <= 16 else "k_spmm_sym"
    print(json.dumps({"kernel": kern, "n": spec.n, "m": m, "x": args.spmm_dtype, "nnz_upper": nnz,
                      "launches": args.steps, "median_ms": round(ms, 4), "algorithmic_bytes": b,
                      "algorithmic_GBps": round(b / ms / 1e6, 1), "copy_bytes_each_way": spec.n * m * es}),
          flush=True)


def warm_start_leg(ctx, M, spec, X0, hnorm, k, nb):
    """Start vectors from a smaller problem (the analogue of the paper's
    N_max - 2 starts, Section 3): the 8 + 2 lowest eigenvectors of the leading
    quarter of H, solved by LOBPCG to 1e-3, padded with zeros, against the
    seeded random start; the benchmark's hybrid and plain LOBPCG.  The warm
    times include the smaller solve."""
    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy
    from paper_2305_15552_amd import warmstart as ws
    ns = spec.n // 4
    brp, bci, bv = sg.gen_block_rows(spec, 0, spec.nbr // 4)
    Ms = hy.matrix_from_csr(ctx, ns, *ws.principal_csr(brp, bci, bv, ns))
    del brp, bci, bv
    out = {"workload": "leading %d x %d principal submatrix solved to 1e-3 (LOBPCG block %d), padded with zeros"
                       % (ns, ns, nb)}
    for name, method in (("hybrid", hy.LOBPCG_RMMDIIS), ("lobpcg", hy.LOBPCG)):
        p = hy.params_default(k=k, nb=nb, method=method, tol=1e-6, hnorm=hnorm, maxiter=3000,
                              switch_rule=hy.SWITCH_RESID, switch_thr=1e-3, s_max=10, rmm_maxiter=300,
                              precision=hy.PREC_F32, precond=hy.PRECOND_JACOBI)
        row = {}
        for start in ("random", "warm"):
            torch.cuda.synchronize()
            t = time.time()
            sub_it = 0
            if start == "warm":
                Xs = X0[:ns].clone()
                ps = hy.params_default(k=k, nb=nb, method=hy.LOBPCG, tol=1e-3, hnorm=hnorm, maxiter=3000,
                                       precision=hy.PREC_F32, precond=hy.PRECOND_JACOBI)
                _, _, reps, _, _ = hy.solve_lowest_k(ctx, Ms, ps, Xs)
                sub_it = reps.iters_front
                X = torch.zeros_like(X0)
                X[:ns] = Xs
            else:
                X = X0.clone()
            ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
            torch.cuda.synchronize()
            row[start] = {"time_s": round(time.time() - t, 4), "status": int(st), "sub_iterations": sub_it,
                          "iterations": [rep.iters_front, rep.iters_rmm, rep.iters_back],
                          "max_resid_hnorm": float(rs.max())}
            log("bench: warm-start leg, %s from %s start: %.3f s, iterations %s (+%d on the submatrix)"
                % (name, start, row[start]["time_s"], row[start]["iterations"], sub_it))
        out[name] = row
    Ms.close()
    return out


def precision_forms_small():
    """The precision forms on the n = 8192 matrix (seed 100): plain FP64, FP32 and
    BF16 stored values (split-BF16 Gram sums, FP32 refinement sweeps after the
    BF16 phase), LOBPCG block 8 to the 8 lowest pairs at 1e-6; eigenvalue errors
    against the dense-eigh spectrum stored with the tests."""
    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy
    gold = os.path.join(ROOT, "tests", "golden", "small_n8192_seed100_spectrum.txt")
    kv = dict(l.split() for l in open(gold) if l.strip() and not l.startswith("#"))
    lam = np.array([float(kv["lambda%d" % (i + 1)]) for i in range(8)])
    hn = float(kv["norm2"])
    spec = sg.SMALL
    rp, ci, v = sg.gen_csr(spec)
    ctx = hy.Context(0)
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v, flags=hy.MAT_BF16)
    X0 = torch.from_numpy(sg.start_block(spec, 8).astype(np.float32)).cuda()
    out = {}
    for name, prec in (("plain_f64", hy.PREC_PLAIN_F64), ("f32", hy.PREC_F32), ("bf16_values", hy.PREC_BF16_SPMM)):
        p = hy.params_default(k=8, nb=8, method=hy.LOBPCG, tol=1e-6, hnorm=hn, maxiter=1000, precision=prec)
        ts = []
        for _ in range(3):
            X = X0.clone()
            torch.cuda.synchronize()
            t = time.time()
            ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
            torch.cuda.synchronize()
            ts.append(time.time() - t)
        err = np.abs(ev - lam) / np.abs(lam)
        out[name] = {"time_s": round(float(np.median(ts)), 4), "status": int(st), "iterations": rep.iters_front,
                     "fp32_refinement_iterations": rep.iters_refine if prec == hy.PREC_BF16_SPMM else None,
                     "max_rel_eig_err_vs_eigh": float(err.max()), "rel_eig_err_vs_eigh": [float(e) for e in err],
                     "max_resid_hnorm": float(rs.max())}
        log("bench: n=8192 %s: %.4f s, %d iterations, max eig err %.2e, max resid %.2e"
            % (name, out[name]["time_s"], rep.iters_front, err.max(), rs.max()))
    M.close()
    ctx.close()
    out["workload"] = ("n=8192 (seed 100) LOBPCG block 8, 8 lowest pairs, tol 1e-6 relative to ||H||_2, shifted "
                       "Jacobi; errors against dense eigh")
    return out


def switch_study_small():
    """The analogue of the paper's Fig. 8 on the n = 8192 matrix (seed 100):
    block Lanczos (block 8) -> RMM-DIIS for the 5 lowest pairs, switching after
    a fixed number of front-end iterations or at tau < 1e-7, with the RMM-DIIS
    product coupled (one product over all 5 columns) or decoupled after c
    converged columns (one SpMV per remaining column).  The cost is the
    effective SpMV count of Section 4.2: the time of all products divided by
    the time of one SpMV on this matrix (cache-resident here, so the ratio is
    that of the cache, not of HBM)."""
    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy
    gold = os.path.join(ROOT, "tests", "golden", "small_n8192_seed100_spectrum.txt")
    kv = dict(l.split() for l in open(gold) if l.strip() and not l.startswith("#"))
    hn = float(kv["norm2"])
    spec = sg.SMALL
    rp, ci, v = sg.gen_csr(spec)
    ctx = hy.Context(0)
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v)
    nnz = int(rp[-1])
    f32 = torch.float32
    prods = product_table(ctx, M, spec, nnz, ((1, f32, f32), (5, f32, f32), (8, f32, f32)), reps=21)
    t1 = prods[0]["median_ms"]
    X0 = torch.from_numpy(sg.start_block(spec, 8).astype(np.float32)).cuda()
    rows = []
    for sw in (10, 20, 30, 40, "tau"):
        for c in (0, 1, 2, 3, 4):
            kw = dict(switch_rule=hy.SWITCH_TAU, switch_thr=1e-7) if sw == "tau" else \
                dict(switch_rule=hy.SWITCH_ITERS, switch_thr=float(sw))
            p = hy.params_default(k=5, nb=8, method=hy.BLANCZOS_RMMDIIS, tol=1e-6, hnorm=hn, maxiter=200,
                                  s_max=10, rmm_maxiter=300, rmm_decouple=c, precision=hy.PREC_F32, **kw)
            X = X0.clone()
            torch.cuda.synchronize()
            t = time.time()
            ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
            torch.cuda.synchronize()
            rows.append({"switch_after": sw if sw != "tau" else "tau<1e-7 (%d)" % rep.iters_front,
                         "rmm_product": "coupled" if c == 0 else "decoupled after %d" % c, "status": int(st),
                         "front": rep.iters_front, "rmm_sweeps": rep.iters_rmm, "lobpcg_after": rep.iters_back,
                         "products": rep.spmm_count, "spmv": rep.spmv_count,
                         "effective_spmv": round(rep.ms_spmm / t1, 1), "time_s": round(time.time() - t, 4)})
    M.close()
    ctx.close()
    log("bench: switch study on n=8192: %d solves" % len(rows))
    return {"workload": "n=8192 (seed 100) block Lanczos(8) -> RMM-DIIS, 5 lowest pairs, tol 1e-6 relative to "
                        "||H||_2; effective SpMV = product time / one SpMV's time (%.4f ms)" % t1,
            "products": prods, "rows": rows}


def methods_small():
    """The analogue of the paper's Tables 4-5 (SpMV counts of the methods for 5
    and 10 pairs) on the n = 8192 matrix (seed 100), with the effective SpMV
    count of Section 4.2 beside them: Lanczos (block size 1), block Lanczos,
    LOBPCG, ChebFSI (degree 10, cutoff at the largest Ritz value) and the three
    hybrids (tau < 1e-7 switch), block 8 for 5 pairs and 16
    for 10, FP32 form, tol 1e-6 relative to ||H||_2.  Counts leave out the final
    FP64 check's product (k SpMVs); the effective count is the solver's product
    time over one SpMV's time on this (cache-resident) matrix."""
    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy
    gold = os.path.join(ROOT, "tests", "golden", "small_n8192_seed100_spectrum.txt")
    kv = dict(l.split() for l in open(gold) if l.strip() and not l.startswith("#"))
    hn = float(kv["norm2"])
    lam = np.array([float(kv["lambda%d" % (i + 1)]) for i in range(10)])
    spec = sg.SMALL
    rp, ci, v = sg.gen_csr(spec)
    ctx = hy.Context(0)
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v)
    nnz = int(rp[-1])
    f32, f64 = torch.float32, torch.float64
    # the final check's product: FP32 vectors, FP64 sums
    prods = product_table(ctx, M, spec, nnz, ((1, f32, f32), (5, f32, f64), (10, f32, f64)), reps=21)
    t1 = prods[0]["median_ms"]
    t_check = {5: prods[1]["median_ms"], 10: prods[2]["median_ms"]}
    rows = []
    for k, nb in ((5, 8), (10, 16)):
        X0 = torch.from_numpy(sg.start_block(spec, nb).astype(np.float32)).cuda()
        for name, method, bsz in (("Lanczos", hy.BLANCZOS, 1), ("block Lanczos", hy.BLANCZOS, nb),
                                  ("LOBPCG", hy.LOBPCG, nb), ("ChebFSI (degree 10)", hy.CHEBFSI, nb),
                                  ("LOBPCG -> RMM-DIIS", hy.LOBPCG_RMMDIIS, nb),
                                  ("block Lanczos -> RMM-DIIS", hy.BLANCZOS_RMMDIIS, nb),
                                  ("ChebFSI -> RMM-DIIS", hy.CHEBFSI_RMMDIIS, nb)):
            p = hy.params_default(k=k, nb=bsz, method=method, tol=1e-6, hnorm=hn, maxiter=1500 if bsz == 1 else 400,
                                  switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, s_max=10, rmm_maxiter=300,
                                  precision=hy.PREC_F32, precond=hy.PRECOND_JACOBI)
            X = torch.zeros((spec.n, max(bsz, k)), dtype=torch.float32, device="cuda")
            X[:, :bsz] = X0[:, :bsz]
            torch.cuda.synchronize()
            t = time.time()
            ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
            torch.cuda.synchronize()
            dt = time.time() - t
            rows.append({"pairs": k, "method": name, "block": bsz, "status": int(st),
                         "spmv": int(rep.spmv_count - k), "products": rep.spmm_count - 1,
                         "effective_spmv": round((rep.ms_spmm - t_check[k]) / t1, 1),
                         "iterations": [rep.iters_front, rep.iters_rmm, rep.iters_back], "time_s": round(dt, 4),
                         "max_rel_eig_err": float(np.max(np.abs(ev - lam[:k]) / np.abs(lam[:k]))),
                         "max_resid_hnorm": float(rs.max())})
            log("bench: methods n=8192 %d pairs, %s: %d SpMVs, %.0f effective, %.3f s, status %d"
                % (k, name, rows[-1]["spmv"], rows[-1]["effective_spmv"], dt, st))
    M.close()
    ctx.close()
    return {"workload": "n=8192 (seed 100), tol 1e-6 relative to ||H||_2, FP32 form, shifted Jacobi for LOBPCG; "
                        "one SpMV %.4f ms" % t1, "rows": rows}


def large_workload(args):
    """The large single-GPU instance: n = 33,554,432 (1,048,576 block rows, 48
    upper tiles per block row within 16384 block rows, p = 0.25, seed 102; about
    1.3e10 stored entries), block Lanczos (block 8) -> RMM-DIIS for the 8 lowest
    pairs, switch at tau < 1e-7 or after 40 front-end iterations (the stored
    Lanczos basis is 1.07 GB per block), LOBPCG with 16 columns if RMM-DIIS
    stagnates.  Reports the product alone at full size (m = 8, 16, 1 and the
    FP64-accumulated form), the solve, and the block Lanczos split between
    products and re-orthogonalisation per iteration."""
    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy
    spec = sg.LARGE
    K, NB, NBB, FRONT = 8, 8, 16, 40
    t0 = time.time()
    rp, ci, v, nnz = sg.device_csr(spec, "cuda:0", chunk=65536, log=log)
    log("bench: generated n=%d nnz=%d on the device in %.1f s" % (spec.n, nnz, time.time() - t0))
    ctx = hy.Context(0)
    t0 = time.time()
    M = hy.Matrix(ctx, spec.n, rp, ci, v, nnz=nnz)
    torch.cuda.synchronize()
    del rp, ci, v
    torch.cuda.empty_cache()
    log("bench: prepared matrix (%d tiles, %.1f GB) in %.1f s" % (M.info.ntiles, M.info.prepared_bytes / 1e9,
                                                                   time.time() - t0))
    f32, f64 = torch.float32, torch.float64
    products = product_table(ctx, M, spec, nnz, ((1, f32, f32), (8, f32, f32), (16, f32, f32), (8, f32, f64)))
    t_spmv = products[0]["median_ms"]
    X0 = torch.from_numpy(sg.start_block(spec, NB).astype(np.float32)).cuda()
    p = hy.params_default(k=1, nb=1, method=hy.LOBPCG, tol=1.0, hnorm=0.0, maxiter=0)
    _, _, rep0, _, _ = hy.solve_lowest_k(ctx, M, p, X0[:, :1].clone())
    hnorm = rep0.hnorm_used
    log("bench: ||H||_2 estimate %.6f" % hnorm)
    params = hy.params_default(k=K, nb=NB, method=hy.BLANCZOS_RMMDIIS, tol=1e-6, hnorm=hnorm, maxiter=FRONT,
                               switch_rule=hy.SWITCH_TAU, switch_thr=1e-7, s_max=10, rmm_maxiter=200,
                               nb_back=NBB, maxiter_back=1500, precision=hy.PREC_F32, precond=hy.PRECOND_JACOBI)

    def solve():
        X = X0.clone()
        torch.cuda.synchronize()
        t = time.time()
        ev, rs, rep, st, hist = hy.solve_lowest_k(ctx, M, params, X, hist_cap=8000)
        torch.cuda.synchronize()
        return time.time() - t, ev, rs, rep, st

    for w in range(args.warmup):
        dt, ev, rs, rep, st = solve()
        log("bench: warmup %d: %.3f s, status %d" % (w, dt, st))
    times, reps = [], []
    t_all = time.time()
    for s_ in range(args.steps):
        dt, ev, rs, rep, st = solve()
        times.append(dt)
        reps.append(rep)
        log("bench: step %d: %.3f s, status %d, iters front %d rmm %d back %d, spmm %d, max resid %.2e"
            % (s_, dt, st, rep.iters_front, rep.iters_rmm, rep.iters_back, rep.spmm_count, rs.max()))
    wall = time.time() - t_all
    t_step = wall / args.steps
    rep = reps[-1]
    # block Lanczos iterations: product time against the rest (re-orthogonalisation
    # against all stored blocks, the three-term recurrence, Cholesky-QR) and the
    # host eigenproblem of the block tridiagonal matrix
    ht = rep.hist_times
    split = []
    for i in range(1, min(rep.iters_front, ht.shape[0])):
        dt_ = ht[i, 0] - ht[i - 1, 0]
        ds = ht[i, 1] - ht[i - 1, 1]
        dsm = ht[i, 2] - ht[i - 1, 2]
        split.append((i + 1, ds, dt_ - ds - dsm, dsm))
    pick = [r for r in split if r[0] in (2, 5, 10, 20, 30, 40)]
    bytes_ = sum(r.bytes_spmm for r in reps)
    ms = sum(r.ms_spmm for r in reps)
    launches = sum(r.spmm_count for r in reps)
    achieved = bytes_ / (ms * 1e6)
    out = {
        "metric": METRIC, "value": round(t_step, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t_step, 2), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": "half-stored symmetric n=33,554,432, 48 upper 32x32 tiles per block row within 16384 "
                        "block rows, p=0.25, seed 102; block Lanczos(8) -> RMM-DIIS, 8 lowest pairs, switch at "
                        "tau<1e-7 or after %d front-end iterations, LOBPCG(%d) on stagnation, shifted Jacobi, "
                        "tol 1e-6 relative to ||H||_2" % (FRONT, NBB),
            "n": spec.n, "nnz_upper": nnz, "k": K, "nb": NB,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_spmm_sym_mma2 at FP32 widths 9-16, k_spmm_sym otherwise (all products of the timed solves)",
            "launches": launches, "avg_ms": round(ms / max(launches, 1), 4),
        },
        "products": products,
        "solve": {
            "eigenvalues": [round(float(x), 10) for x in ev], "max_resid_hnorm": float(rs.max()),
            "orth_err": rep.orth_err, "status": int(st), "iters_front": rep.iters_front,
            "iters_rmm": rep.iters_rmm, "iters_back": rep.iters_back, "spmm_count": rep.spmm_count,
            "switched": rep.switched, "fallback_used": rep.fallback_used, "ms_spmm": round(rep.ms_spmm, 1),
            "spmv_count": rep.spmv_count, "effective_spmv": round(rep.ms_spmm / t_spmv, 1),
            "ms_small": round(rep.ms_small, 1), "ms_dense_and_sync": round(rep.ms_dense, 1),
            "step_times_s": [round(t, 3) for t in times],
        },
        "block_lanczos_split": [{"iteration": i, "product_ms": round(a, 2), "reorth_and_rest_ms": round(b, 2),
                                 "tridiag_eig_ms": round(c, 2), "ratio_to_product": round(b / a, 3)}
                                for i, a, b, c in pick],
    }
    # no oracle baseline at this size: the oracle's product holds U and its transpose in host memory (about
    # 210 GB here, beside the generator's arrays), and no oracle reference run fixes its iteration count
    out["cpu_baseline"] = None
    out["cpu_baseline_note"] = ("not run for n = 33,554,432: the FP64 oracle's product needs both triangles in "
                                "host memory (about 210 GB) and no oracle reference run exists at this size; the "
                                "default workload (n = 2,097,152) reports it")
    print(json.dumps(out), flush=True)


def mlp_leg(ctx, M, spec, hnorm, lam_gold):
    """Learned preconditioner on this matrix (seed 101, not a training seed): the
    MLP is trained by the library on samples from n=8192 generator matrices
    (seeds 0-7).  Three arms run LOBPCG (block 16) to the lowest 8 pairs at 1e-6
    from the same three start blocks: the plain FP64 form with the shifted
    diagonal, the FP32 form with the shifted diagonal, the FP32 form with the
    MLP.  Reported per arm: iterations and time to solution for each start block,
    their mean, minimum and maximum."""
    import numpy as np
    import synthgen as sg
    import torch
    from paper_2305_15552_amd import hyeig as hy
    from paper_2305_15552_amd import learned
    t0 = time.time()
    mats = []
    for seed in range(8):
        sp = sg.MatrixSpec(8192, 15, 64, 0.25, seed)
        rp, ci, v = sg.gen_csr(sp)
        Mt = hy.matrix_from_csr(ctx, sp.n, rp, ci, v, flags=hy.MAT_ROWSTATS)
        mats.append((Mt, torch.from_numpy(sg.start_block(sp, 8).astype(np.float32)).cuda()))
    F, T = learned.collect_samples(ctx, mats)
    torch.cuda.synchronize()
    t1 = time.time()
    mlp, losses = learned.train(ctx, F, T, epochs=20, batch=65536, lr=1e-3, clip=100.0)
    torch.cuda.synchronize()
    t2 = time.time()
    for Mt, _ in mats:
        Mt.close()
    stream = ctx.stream
    # inference alone (hyeig_mlp_forward): the samples tiled to 2^24, timed with
    # events on the library context's stream; 640 FLOP and 20 bytes (4 features
    # in, 1 output) per sample
    reps_ = (1 << 24) // F.shape[0] + 1
    Fb = F.repeat(reps_, 1)[: 1 << 24].contiguous()
    ob = torch.empty(Fb.shape[0], dtype=torch.float32, device="cuda")
    mlp.forward(Fb, ob)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        mlp.forward(Fb, ob)
    e1.record(stream)
    torch.cuda.synchronize()
    inf_s = e0.elapsed_time(e1) / 1e3 / 10
    ns = Fb.shape[0]
    del Fb, ob
    # the apply as LOBPCG calls it, on an n x 16 FP32 residual block: the whole
    # hyeig_mlp_precond call (its column norms, the network on every entry, the
    # non-finite check), host clock around synchronised calls
    Wb = torch.randn(spec.n, 16, dtype=torch.float32, device="cuda")
    th16 = np.linspace(-10.6, -10.0, 16)
    mlp.precond(M, Wb, th16, hnorm)
    torch.cuda.synchronize()
    ta = time.time()
    for _ in range(10):
        mlp.precond(M, Wb, th16, hnorm)
    torch.cuda.synchronize()
    apply_s = (time.time() - ta) / 10
    del Wb
    res = {"inference": {"samples": ns, "ms": round(inf_s * 1e3, 3), "samples_per_s": round(ns / inf_s, 1),
                         "TFLOPs": round(640.0 * ns / inf_s / 1e12, 2), "GBps": round(20.0 * ns / inf_s / 1e9, 1),
                         "frac_bf16_mfma_peak": round(640.0 * ns / inf_s / 2.5e15, 5),
                         "frac_hbm": round(20.0 * ns / inf_s / 8e12, 4)},
           "apply": {"ms": round(apply_s * 1e3, 3), "rows": spec.n, "columns": 16, "dtype": "f32",
                     "what": "one hyeig_mlp_precond call: column norms, network on every entry, rescale, "
                             "non-finite check (host clock, synchronised)"},
           "train": {"samples": int(F.shape[0]), "label_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
                     "train_samples_per_s": round(20 * F.shape[0] / max(t2 - t1, 1e-9), 1),
                     "epochs": 20, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                     "data": "LOBPCG snapshots (2,4,8,16,32 iterations) on n=8192 generator matrices, seeds 0-7; "
                             "targets from 20 GPU MINRES steps on the projected correction equation"}}
    del F, T
    arms = (("plain_f64_jacobi", hy.PREC_PLAIN_F64, hy.PRECOND_JACOBI, None),
            ("f32_jacobi", hy.PREC_F32, hy.PRECOND_JACOBI, None),
            ("f32_mlp", hy.PREC_F32, hy.PRECOND_MLP, mlp))
    seeds = (spec.seed + 1, spec.seed + 2, spec.seed + 3)
    X0s = [torch.from_numpy(sg.normal_block(spec.n, 16, s, 4).astype(np.float32)).cuda() for s in seeds]

    def run(prec, pk, m, X0, maxiter=3000):
        p = hy.params_default(k=8, nb=16, method=hy.LOBPCG, tol=1e-6, hnorm=hnorm, maxiter=maxiter,
                              precision=prec, precond=pk, mlp=m)
        X = X0.clone()
        torch.cuda.synchronize()
        t = time.time()
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, p, X)
        torch.cuda.synchronize()
        return time.time() - t, ev, rs, rep, st

    for name, prec, pk, m in arms:  # untimed: first calls of each form
        run(prec, pk, m, X0s[0], maxiter=3)
    out = {}
    for name, prec, pk, m in arms:
        r = {"iterations": [], "time_s": [], "status": [], "max_resid_hnorm": [], "max_rel_eig_err": [],
             "mlp_fallbacks": []}
        for s, X0 in zip(seeds, X0s):
            dt, ev, rs, rep, st = run(prec, pk, m, X0)
            r["iterations"].append(rep.iters_front)
            r["time_s"].append(round(dt, 4))
            r["status"].append(int(st))
            r["max_resid_hnorm"].append(float(rs.max()))
            r["max_rel_eig_err"].append(float(np.max(np.abs(ev[:8] - lam_gold[:8]) / np.abs(lam_gold[:8])))
                                        if lam_gold is not None else None)
            r["mlp_fallbacks"].append(rep.events_mlp_fallback)
            log("bench: learned-preconditioner leg, %s, X0 seed %d: %d iterations, %.3f s, status %d"
                % (name, s, rep.iters_front, dt, st))
        for key in ("iterations", "time_s"):
            v = np.asarray(r[key], dtype=float)
            r[key + "_mean"] = round(float(v.mean()), 4)
            r[key + "_min"] = round(float(v.min()), 4)
            r[key + "_max"] = round(float(v.max()), 4)
        r["ms_per_iteration"] = round(1e3 * sum(r["time_s"]) / max(sum(r["iterations"]), 1), 3)
        out[name] = r
    res["arms"] = out
    res["X0_seeds"] = list(seeds)
    res["speedup_f32_mlp_vs_plain_f64_jacobi"] = round(out["plain_f64_jacobi"]["time_s_mean"]
                                                       / out["f32_mlp"]["time_s_mean"], 3)
    res["speedup_f32_mlp_vs_f32_jacobi"] = round(out["f32_jacobi"]["time_s_mean"] / out["f32_mlp"]["time_s_mean"], 3)
    # what the network's apply adds to a FP32 iteration, over the shifted diagonal
    res["apply_ms_per_iteration_in_solver"] = round(out["f32_mlp"]["ms_per_iteration"]
                                                    - out["f32_jacobi"]["ms_per_iteration"], 3)
    res["workload"] = ("n=2,097,152 generator matrix (seed 101), LOBPCG block 16, lowest 8 pairs, tol 1e-6 relative "
                       "to ||H||_2, start blocks N(0,1) with seeds 102-104")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-chosen", action="store_true", help="skip the chosen FP32 form beside the plain one")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm start from the principal submatrix")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the precision forms and the switch study on the n=8192 matrix")
    ap.add_argument("--workload", choices=["scale", "large"], default="scale",
                    help="scale: n=2,097,152 hybrid LOBPCG->RMM-DIIS (default); large: n=33,554,432 block "
                         "Lanczos->RMM-DIIS (about 2 minutes of host generation, 225 GB of device memory)")
    ap.add_argument("--spmm-only", action="store_true",
                    help="time only the product (width --spmm-width, x and sums --spmm-dtype) and a plain copy of "
                         "known size, for profiling")
    ap.add_argument("--spmm-dtype", choices=["f32", "f64"], default="f64",
                    help="x and accumulation type of --spmm-only (f64: the plain form's product)")
    ap.add_argument("--spmm-width", type=int, default=16,
                    help="block width of --spmm-only (16: matrix-core kernel; 8: the tile walk)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; runs on %d GPUs are not part of it" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synthgen as sg
    from paper_2305_15552_amd import hyeig as hy

    if args.workload == "large":
        return large_workload(args)
    spec = sg.SCALE
    K, NB = 10, 16
    if args.spmm_only:
        return spmm_only(spec, args.spmm_width, args)
    t0 = time.time()
    rp, ci, v = sg.gen_csr(spec)
    nnz = int(rp[-1])
    log("bench: generated n=%d nnz=%d in %.1f s" % (spec.n, nnz, time.time() - t0))
    ctx = hy.Context(0)
    t0 = time.time()
    M = hy.matrix_from_csr(ctx, spec.n, rp, ci, v, flags=hy.MAT_BF16 | hy.MAT_ROWSTATS)
    del rp, ci, v
    log("bench: prepared matrix (%d tiles) in %.1f s" % (M.info.ntiles, time.time() - t0))
    X0 = torch.from_numpy(sg.start_block(spec, NB).astype(np.float32)).cuda()

    # ||H||_2 once, by the library's 30-step Lanczos estimate (outside the timed region)
    p = hy.params_default(k=1, nb=1, method=hy.LOBPCG, tol=1.0, hnorm=0.0, maxiter=0)
    Xt = X0[:, :1].clone()
    _, _, rep0, _, _ = hy.solve_lowest_k(ctx, M, p, Xt)
    hnorm = rep0.hnorm_used
    log("bench: ||H||_2 estimate %.6f" % hnorm)

    def params(prec):
        return hy.params_default(k=K, nb=NB, method=hy.LOBPCG_RMMDIIS, tol=1e-6, hnorm=hnorm, maxiter=2000,
                                 switch_rule=hy.SWITCH_RESID, switch_thr=1e-3, s_max=10, rmm_maxiter=300,
                                 precision=prec, precond=hy.PRECOND_JACOBI)

    def solve(prec, hist_cap=0):
        X = X0.clone()
        torch.cuda.synchronize()
        t = time.time()
        ev, rs, rep, st, _ = hy.solve_lowest_k(ctx, M, params(prec), X, hist_cap=hist_cap)
        torch.cuda.synchronize()
        return time.time() - t, ev, rs, rep, st

    gold = golden_scale()
    lam_gold = np.array([float(gold["lambda%d" % (i + 1)]) for i in range(K)]) if gold else None

    def eig_err(ev):
        return float(np.max(np.abs(np.asarray(ev) - lam_gold) / np.abs(lam_gold))) if gold else None

    # the headline: the plain FP64 form (FP64 blocks and sums, the paper's arithmetic)
    for w in range(args.warmup):
        dt, ev, rs, rep, st = solve(hy.PREC_PLAIN_F64)
        log("bench: warmup %d: %.3f s, status %d, iters %d/%d/%d" % (w, dt, st, rep.iters_front, rep.iters_rmm,
                                                                      rep.iters_back))
    times, reps = [], []
    torch.cuda.synchronize()
    t_all = time.time()
    for s_ in range(args.steps):
        dt, ev, rs, rep, st = solve(hy.PREC_PLAIN_F64, hist_cap=8000)
        times.append(dt)
        reps.append(rep)
        log("bench: step %d: %.3f s, status %d, iters front %d rmm %d back %d, spmm %d, max resid %.2e"
            % (s_, dt, st, rep.iters_front, rep.iters_rmm, rep.iters_back, rep.spmm_count, rs.max()))
        if st != hy.OK:
            log("bench: solve did not reach the tolerance")
    torch.cuda.synchronize()
    wall = time.time() - t_all
    t_step = wall / args.steps
    rep = reps[-1]
    # the product alone at the widths the solves use and at width 1 (SpMM/SpMV ratio), both forms
    f32, f64 = torch.float32, torch.float64
    products = product_table(ctx, M, spec, nnz, ((1, f64, f64), (8, f64, f64), (16, f64, f64),
                                                 (1, f32, f32), (8, f32, f32), (10, f32, f32), (16, f32, f32)))
    t_spmv = products[0]["median_ms"]
    # roofline of the dominant kernel (the FP64 product on matrix cores) from the in-solve HIP events of its
    # own launches; all products of the solves beside it
    bytes_ = sum(r.bytes_spmm_mc for r in reps)
    ms = sum(r.ms_spmm_mc for r in reps)
    launches = sum(r.spmm_mc_count for r in reps)
    achieved = bytes_ / (ms * 1e6)  # GB/s
    all_b = sum(r.bytes_spmm for r in reps)
    all_ms = sum(r.ms_spmm for r in reps)
    all_n = sum(r.spmm_count for r in reps)
    copy_gbs = copy_bandwidth()
    ht = rep.hist_times
    cond_trace = [{"iteration": i, "cond_StS": float(ht[i, 3])}
                  for i in (1, 2, 5, 10, 20, 40, 60, 80, rep.iters_front) if 0 < i <= rep.iters_front
                  and i < ht.shape[0]]
    out = {
        "metric": METRIC,
        "value": round(t_step, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "half-stored symmetric n=2,097,152, 24 upper 32x32 tiles per block row within 4096 "
                        "block rows, p=0.3, seed 101; hybrid LOBPCG(16)->RMM-DIIS, 10 lowest pairs, switch at "
                        "residual 1e-3, shifted Jacobi, tol 1e-6 relative to ||H||_2; plain FP64 form",
            "n": spec.n, "nnz_upper": nnz, "k": K, "nb": NB,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counted_traffic(),
            "kernel": "k_spmm_sym_mma2<double, double> (FP64 matrix cores, widths 9-16): its launches in the timed "
                      "plain FP64 solves",
            "launches": launches, "avg_ms": round(ms / max(launches, 1), 4),
            "traffic_per": "launch at m = 16 (L2-miss bytes, calibrated FETCH_SIZE + WRITE_SIZE)",
            "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
            "all_products": {"launches": all_n, "avg_ms": round(all_ms / max(all_n, 1), 4),
                             "achieved_GBps": round(all_b / (all_ms * 1e6), 1),
                             "what": "every product of the timed solves, the tile walk's narrow ones included"},
        },
        "solve": {
            "form": "plain FP64: FP64 blocks, FP64 sums in every product, FP32 stored values (the matrix)",
            "eigenvalues": [round(float(x), 10) for x in ev],
            "max_rel_eig_err_vs_oracle": eig_err(ev),
            "max_resid_hnorm": float(rs.max()), "max_resid_theta": rep.resid_theta_max,
            "orth_err": rep.orth_err, "iters_front": rep.iters_front, "iters_rmm": rep.iters_rmm,
            "iters_back": rep.iters_back, "spmm_count": rep.spmm_count, "spmv_count": rep.spmv_count,
            "fallback_used": rep.fallback_used, "merged_back": rep.merged_back, "ms_spmm": round(rep.ms_spmm, 2), "ms_small": round(rep.ms_small, 2),
            "effective_spmv": round(rep.ms_spmm / t_spmv, 1),
            "ms_dense_and_sync": round(rep.ms_dense, 2), "converged": bool(rep.converged),
            "step_times_s": [round(t, 4) for t in times],
            "max_cond_StS": rep.max_cond, "cond_trace": cond_trace,
        },
        "products": products,
    }
    if gold:
        out["solve"]["oracle_reference"] = ("tests/golden/scale_n2097152_seed101_spectrum.txt (FP64 oracle, two "
                                            "LOBPCG routes agreeing to 1e-10)")
    if not args.no_chosen:
        # the chosen form beside it: FP32 blocks and sums, FP64 small problems and final check
        ct, crep = [], None
        for _ in range(max(1, min(args.steps, 5))):
            dtc, evc, rsc, crep, stc = solve(hy.PREC_F32)
            ct.append(dtc)
        tc = float(np.median(ct))
        log("bench: chosen FP32 form: %.3f s (median of %d), status %d, iters %d/%d/%d" % (
            tc, len(ct), stc, crep.iters_front, crep.iters_rmm, crep.iters_back))
        cb = crep.bytes_spmm_mc / (crep.ms_spmm_mc * 1e6)
        out["chosen_f32"] = {
            "form": "FP32 blocks and FP32 sums in the products (matrix cores at widths 9-16), FP64 Gram sums, "
                    "small problems and final check",
            "time_s": round(tc, 4), "step_times_s": [round(t, 4) for t in ct], "status": int(stc),
            "max_resid_hnorm": float(rsc.max()), "max_rel_eig_err_vs_oracle": eig_err(evc),
            "max_rel_eig_diff_vs_plain": float(np.max(np.abs(evc - ev) / np.abs(ev))),
            "iters_front": crep.iters_front, "iters_rmm": crep.iters_rmm, "iters_back": crep.iters_back,
            "spmm_count": crep.spmm_count, "ms_spmm": round(crep.ms_spmm, 2), "ms_small": round(crep.ms_small, 2),
            "ms_dense_and_sync": round(crep.ms_dense, 2),
            "spmm_avg_ms": round(crep.ms_spmm / max(crep.spmm_count, 1), 4),
            "spmm_roofline": {"bound": "hbm", "achieved": round(cb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(cb / HBM_PEAK_GBS, 4),
                              "traffic": counted_traffic("spmm_mma_c2_m16_hbm_counters.txt"),
                              "kernel": "k_spmm_sym_mma2<float, float> (FP32 matrix cores, widths 9-16): its "
                                        "launches in the timed FP32 solves",
                              "launches": crep.spmm_mc_count,
                              "avg_ms": round(crep.ms_spmm_mc / max(crep.spmm_mc_count, 1), 4)},
        }
        out["speedup_chosen_vs_plain"] = round(t_step / tc, 3)
    if not args.no_mlp:
        out["learned_preconditioner"] = mlp_leg(ctx, M, spec, hnorm, lam_gold)
    if not args.no_warm:
        out["warm_start"] = warm_start_leg(ctx, M, spec, X0, hnorm, K, NB)
    if not args.no_small:
        out["precision_forms_small"] = precision_forms_small()
        out["switch_study_small"] = switch_study_small()
        out["methods_small"] = methods_small()
    if not args.no_cpu:
        M.close()
        torch.cuda.empty_cache()
        try:
            out["cpu_baseline"] = cpu_baseline(spec, NB, K, hnorm)
        except MemoryError:
            out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
