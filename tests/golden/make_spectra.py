"""Writes the exact low spectrum of the n=8192 test matrix (seed 100) with
dense LAPACK eigh through the oracle.  Calls only oracle/ and synthgen/.

    python tests/golden/make_spectra.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synthgen as sg  # noqa: E402
from oracle.sparse import HalfSym  # noqa: E402


def main():
    spec = sg.SMALL
    H = HalfSym(spec.n, *sg.gen_csr(spec))
    w = np.linalg.eigvalsh(H.dense())
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_n8192_seed100_spectrum.txt")
    with open(out, "w") as f:
        f.write("# exact eigenvalues of the n=8192 synthetic matrix (t=15, w=64, p=0.25, seed 100)\n")
        f.write("# dense numpy.linalg.eigh of the oracle's H = U + U^T - diag(U); written by make_spectra.py\n")
        f.write("norm2 %.17g\n" % max(abs(w[0]), abs(w[-1])))
        for i in range(32):
            f.write("lambda%d %.17g\n" % (i + 1, w[i]))
        f.write("lambda_max %.17g\n" % w[-1])


if __name__ == "__main__":
    main()
