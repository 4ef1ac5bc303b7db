"""The C-ABI library loads and exports every function include/hyeig.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyeig.h")
LIB = os.path.join(ROOT, "paper_2305_15552_amd", "libhyeig.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hyeig_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for want in ["hyeig_spmm_sym", "hyeig_gram", "hyeig_block_update", "hyeig_cholqr", "hyeig_rayleigh_ritz",
                 "hyeig_rmm_diis_step", "hyeig_solve_lowest_k", "hyeig_mlp_forward", "hyeig_mlp_backward",
                 "hyeig_mlp_train"]:
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhyeig.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert getattr(lib, n) is not None
