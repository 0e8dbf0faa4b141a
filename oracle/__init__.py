"""Plain FP64 CPU oracle for the KSVD tensor-product block-Jacobi preconditioner.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never
calls, links or falls back to anything here, and nothing here imports the GPU
package.

Each function computes its result by the plain definition it cites in
Pazner & Persson, "Approximate tensor-product preconditioners for very high
order discontinuous Galerkin methods" (arXiv 1704.04549): full SVDs, dense
Kronecker products and dense LU solves, not the fast algorithms.  The one
exception is ``apply.schur_solve``, the paper's own Schur/Sylvester route
(Algs. 5-8), kept as an independent fast CPU path and checked against the
dense definition.

Parity status of each module is stated in its header.
"""
