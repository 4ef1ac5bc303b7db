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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhyeig.so not built")
def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the same size and field
    offsets as the C compiler gives them."""
    torch = pytest.importorskip("torch")  # the binding loads the HIP runtime through torch
    from paper_2305_15552_amd import hyeig as hy
    structs = {"hyeig_params": hy.Params, "hyeig_report": hy.Report, "hyeig_mat_info": hy.MatInfo,
               "hyeig_train_params": hy.TrainParams}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hyeig.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, c = l.split()
        got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhyeig.so not built")
def test_ctypes_structures_match_the_header(tmp_path):
    """The binding's ctypes mirrors of the header's structs: every field at the
    offset a C compiler gives it, and the same total size (a field added on one
    side only would shift the rest without an error)."""
    from paper_2305_15552_amd import hyeig as hy
    pairs = [("hyeig_params", hy.Params), ("hyeig_report", hy.Report), ("hyeig_mat_info", hy.MatInfo),
             ("hyeig_train_params", hy.TrainParams)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hyeig.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.splitlines())
    for cname, cls in pairs:
        assert int(got[cname + " size"]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(cls, fname).offset, (cname, fname)
