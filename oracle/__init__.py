"""Plain FP64 CPU oracle for the Vanka-type multigrid solve of complex-shifted
Laplacian systems and the ParaDIAG time transform around it.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call,
link or execute anything in this package: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it.  It shares no code, tables or constants with the HIP library.

The code is deliberately slow and literal: NumPy complex128 arrays, no
blocking, no fusion, no reordering beyond what the paper's definitions state.
Each function cites the passage of He & Liu, "A Vanka-type multigrid solver
for complex-shifted Laplacian systems from diagonalization-based
parallel-in-time algorithms" (arXiv 2203.11154) that it follows.

Modules
-------
operators   5-point shifted Laplacian, Vanka patch stencil, transfers
multigrid   V/W cycles, coarsest-grid direct solve, stopping rule
exact       closed-form eigenpairs, DST-I fast exact solve, dense solve
spectral    time-discretisation matrices and their eigen-decompositions
lfa         local / rigorous Fourier analysis (smoothing and two-grid factors)
paradiag    all-at-once heat problem, ParaDIAG-II iteration, adjoint

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
value the paper prints or a fact of the mathematics, except where a
function's docstring says "parity unpinned".
"""
