"""Plain FP64 CPU oracle for the spectral two-level PCG solve.

Test infrastructure only. Nothing in the product path imports it: only the
tests, the smoke check and the benchmark's CPU-baseline leg may call it. It
shares no code with the GPU library; both draw inputs from the seeded
generators in ``paper_1411_3923_amd.workloads`` and nothing else.

Every routine is the definition in the paper written out in numpy/scipy,
double precision, with no blocking, fusion or reordering:

* ``fem``      element stiffness (Sec. 2.1), SIMP (Sec. 2.2, eq. of K_e),
               assembly, direct solve, compliance and its sensitivities
               (Sec. 4.2).
* ``density``  density filter and smoothed Heaviside projection with their
               chain rule (Sec. 4.3), three thresholds (Sec. 4.4).
* ``schwarz``  the spectral coarse space (Sec. 2.4: local generalised
               eigenproblems weighted by diag(K), Sec. 3.2; partition of unity;
               Galerkin coarse matrix) and the two-level additive Schwarz
               preconditioner used inside PCG (Sec. 2.4.2).
"""
