"""CPU oracle for the all-at-once quasi-boundary-value system of Majumdar,
Serra-Capizzano and Sormani, "Block triangular preconditioning for inverse
source problems in time-space fractional diffusion equations" (arXiv
2507.02809).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, FP64 statement of
what the GPU library computes, written from the paper and checked against
what the paper and mathematics fix (closed forms, invariants, the paper's
printed condition numbers and iteration counts).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with ``paper_2507_02809_amd`` (the GPU path); the
only module both sides use is the seeded input generator
``paper_2507_02809_amd.inputs``, which holds none of the method's arithmetic.

Modules
-------
coeffs    L1 weights b_m, e_m, the scaling eta, fractional-Laplacian stencil
          a_l (1D closed form; d-D by a subordination integral), the tau
          symbol.                                            (paper §4, §5)
system    Problem container, dense B, A, P, z, A-hat, z-hat.  (paper §5)
matfree   Matrix-free products: the paper's FFT matvec, forward substitution
          for P (dense-block or CG inner solves), forward problem.
krylov    Textbook GMRES (no / left / right preconditioning) and flexible
          GMRES, used as reference solvers.

Parity status: every function here is pinned by a ``-m "not gpu"`` test,
except where its docstring says "parity unpinned".
"""
