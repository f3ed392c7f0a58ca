"""FP64 CPU oracle for Nys-IP-PMM on the separable QP (P)/(D).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
calls this package; it is used by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  It shares
no code with the HIP library: it is plain numpy/scipy in float64, written
from the paper's definitions and algorithms, slow and direct on purpose.

Modules
-------
problem    definitions of (P)/(D): objectives, KKT residuals, stopping measure
normal_eq  the regularised normal-equation operator and the Newton step
nystrom    randomized Nystrom approximation and the Nystrom preconditioner
pchol      partial Cholesky preconditioner (the Chol-IP-PMM comparator)
boxqp      IP-PMM with free, non-negative and box-constrained variables
portfolio  the factor-model portfolio problem in its original form; brute force
pcg        textbook preconditioned conjugate gradients
ippmm      the IP-PMM outer loop with an exact (dense Cholesky) inner solve
bruteforce active-set enumeration of the KKT conditions of tiny problems
adaptive   sketch size from the effective dimension; reuse rule
adjoint    gradient of a loss of the solution through the KKT conditions
lowprec    round-to-nearest-even emulation of BF16 / FP32 storage
philox     the Philox4x32-10 counter-based generator and Box-Muller normals

Parity status: every function is pinned by a CPU test against something
other than itself (closed forms, invariants, brute force, textbook routines,
published known-answer vectors, or cases worked by hand in exact rational
arithmetic).  The readings that shape the trajectory (initial point,
parameter update, stopping measure) are pinned that way too: hand-derived
initial points and stopping measures, and the parameter update against the
properties the paper states for it.  What stays unpinned is agreement of
iteration counts with the paper's own runs, whose data are not available.
"""
