"""MI355X (gfx950) solver for the quasi-boundary-value inverse source problem of a
time-space fractional diffusion equation: preconditioned GMRES on the all-at-once
system with the block lower-triangular preconditioner (arXiv 2507.02809, §5).

The compute path is the C-ABI library ``libtsfde.so`` (hand-written HIP kernels);
``paper_2507_02809_amd.tsfde`` is a thin ctypes binding to it.  ``inputs`` holds
the seeded synthetic input generator.  Importing this package loads nothing:
``tsfde`` loads the shared library on first use and raises if it is missing.
"""
