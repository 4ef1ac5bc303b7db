"""Writes the ten lowest eigenvalues of the n=2,097,152 workload matrix (seed 101)
with the FP64 oracle, by two independent routes that must agree.  Calls only
oracle/ and synthgen/.

    python tests/golden/make_c2_spectrum.py            (about an hour on 8 host cores)

Route A: oracle LOBPCG (Alg. 2) with block 16 from the seeded start block.
Route B: oracle LOBPCG with block 24 from an unrelated seeded normal block.
Both run in FP64 with the shifted-diagonal preconditioner to a relative
residual of 1e-9 against ||H||_2 (a thousand times tighter than the solver's
1e-6), so the Kato-Temple bound ||r||^2 / gap puts each Ritz value within
~1e-14 of an eigenvalue.  Two block sizes from unrelated starts landing on the
same ten values to 1e-10 is the check that none of the lowest ten was missed.
||H||_2 is the largest |Ritz value| of a 120-step Lanczos run (the spectrum's
upper end; its lower end is the wanted cluster).  The products run on all host
threads through the oracle's plain C loop (oracle/halfsym_omp.c).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synthgen as sg  # noqa: E402
from oracle import solvers  # noqa: E402
from oracle.sparse import HalfSymOMP  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "scale_n2097152_seed101_spectrum.txt")
K = 10
TOL = 1e-9


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def main():
    spec = sg.SCALE
    t0 = time.time()
    rp, ci, v = sg.gen_csr(spec)
    H = HalfSymOMP(spec.n, rp, ci, v)
    del rp, ci, v
    threads = H.nthreads()
    log("matrix n=%d nnz=%d, %d threads, %.1f s" % (spec.n, int(H.rowptr[-1]), threads, time.time() - t0))

    t0 = time.time()
    low, up = solvers.lanczos_norm_estimate(H, spec.n, steps=120)
    hn = low
    log("||H||_2: %.15g (upper estimate %.15g), %.1f s" % (low, up, time.time() - t0))

    routes = {}
    for name, nb, X0 in (("A", 16, sg.start_block(spec, 16)),
                         ("B", 24, sg.normal_block(spec.n, 24, 20240601, stream=5))):
        t0 = time.time()
        it_log = []

        def stop(it, theta, rel, it_log=it_log):
            if it % 10 == 0:
                log("route %s iteration %d: max residual %.3e" % (name, it, float(np.max(rel[:K]))))
            it_log.append(it)
            return False

        r = solvers.lobpcg(H, X0, K, tol=TOL, maxiter=4000, hnorm=hn, precond="jacobi", d=H.d, stop=stop)
        dt = time.time() - t0
        th, rh, _, orth = solvers.final_check(H, r.X[:, :K], hn)
        log("route %s: converged %s, %d iterations, %d products, %.0f s, max final residual %.2e, orth %.1e"
            % (name, r.converged, r.iters, r.spmm, dt, float(rh.max()), orth))
        if not r.converged or rh.max() > TOL:
            raise SystemExit("route %s did not reach the tolerance" % name)
        # the first iteration at which the leading K residuals all reach the solver's 1e-6
        hit = [i for i, h in enumerate(r.history) if np.max(h) <= 1e-6]
        routes[name] = dict(theta=np.sort(th), iters=r.iters, spmm=r.spmm, spmv=r.spmv, secs=dt,
                            resid=float(rh.max()), it6=hit[0] if hit else -1)

    a, b = routes["A"]["theta"], routes["B"]["theta"]
    agree = float(np.max(np.abs(a - b) / np.abs(a)))
    log("routes agree to %.2e relative" % agree)
    if agree > 1e-10:
        raise SystemExit("routes disagree: %.3e" % agree)
    with open(OUT, "w") as f:
        f.write("# ten lowest eigenvalues of the n=2,097,152 synthetic matrix (t=24, w=4096, p=0.3, seed 101)\n")
        f.write("# FP64 oracle, two routes (LOBPCG block 16 from the seeded start block, LOBPCG block 24 from\n")
        f.write("# another seeded block) to relative residual %.0e against norm2; written by make_c2_spectrum.py\n"
                % TOL)
        f.write("# routes agree to %.3e relative; products in FP64 on %d host threads\n" % (agree, threads))
        for nm in ("A", "B"):
            r = routes[nm]
            f.write("# route %s: %d iterations (%d to 1e-6), %d products, %d SpMVs, %.0f s, max residual %.3e\n"
                    % (nm, r["iters"], r["it6"], r["spmm"], r["spmv"], r["secs"], r["resid"]))
        f.write("norm2 %.17g\n" % hn)
        f.write("norm2_upper %.17g\n" % up)
        f.write("oracle_iters %d\n" % routes["A"]["iters"])
        f.write("oracle_iters_to_1e-6 %d\n" % routes["A"]["it6"])
        f.write("oracle_products %d\n" % routes["A"]["spmm"])
        f.write("oracle_spmv %d\n" % routes["A"]["spmv"])
        f.write("oracle_seconds %.1f\n" % routes["A"]["secs"])
        f.write("oracle_threads %d\n" % threads)
        for i in range(K):
            f.write("lambda%d %.17g\n" % (i + 1, a[i]))
    log("wrote", OUT)


if __name__ == "__main__":
    main()
