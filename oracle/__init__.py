"""Plain FP64 CPU oracle for the hybrid eigensolver hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here.  The GPU
library shares no code with this package (no kernels, headers, helpers or
constants); both sides read their inputs from ``synthgen`` only.

Everything is computed in float64 with numpy / scipy.  Each function states
the passage of arXiv 2305.15552 ("Hybrid Eigensolvers for Nuclear
Configuration Interaction Calculations") it follows.  Where the paper leaves a
point open, the function's docstring states the reading it takes.

Modules
  sparse    half-stored symmetric product and the dense block kernels
  dense     small FP64 problems: CholeskyQR, Rayleigh-Ritz, DIIS, 2x2 pencil
  solvers   LOBPCG, block Lanczos, batched RMM-DIIS, hybrid, switch metric
  mlp       FP64 per-row MLP preconditioner, gradients, features, labels

Pins: every function is checked by ``tests/test_oracle_*.py`` against
something other than itself (dense LAPACK eigh, closed forms, brute force,
invariants, worked numbers from the paper).  Functions without such a pin say
"parity unpinned" in their docstring.
"""
