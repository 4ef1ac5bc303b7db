"""The C-ABI from a C program alone (tests/c_abi_demo.c: HIP allocation, the
header and the library, no Python or torch on its side): a product against the
host's and the 4 lowest eigenpairs of tridiag(-1, 2, -1) against the closed
form 2 - 2 cos(j pi / (n + 1))."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi_demo")


def test_c_program_uses_the_library():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "tests/c_abi_demo is not built (__graft_entry__.build())"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "product: max |error|" in r.stdout and "solve:" in r.stdout
