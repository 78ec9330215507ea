"""FP64 CPU oracle for the finite-element Bloch-Torrey time stepping.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link
or execute this package: only the test suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark use it. It shares no code,
tables or helpers with the GPU library; the only thing both consume is the
seeded synthetic input arrays.

What it computes (plain, slow, obviously correct):

* ``sequence``: the PGSE profile f, its integral F, the b-value integral
  and the b -> gradient conversion (Sec. 2, eq. pgse and eq. b_value).
* ``fem``: P1 assembly on a tetrahedral mesh with one field per compartment
  (PUFEM, Appendix A, eq. phase_func), periodic identification of opposite
  box faces (strong pseudo-periodic imposition, Appendix A), and the
  permeable-interface face terms (Sec. 2, eq. btpde_ic).
* ``timestep``: the theta-method recurrence (Appendix A,
  eq. theta_discretization; Appendix B, eq. matrix_form) with an exact sparse
  direct solve (SuperLU) per time step, and the signal at echo time
  (Sec. 2, eq. signal).
* ``mf1d``: a matrix-formalism reference signal for a 1-D slab (the kind of
  reference the paper validates against, Sec. 4), used only as a pin.
* ``mlp``: NumPy forward/backward of the small per-node network used for the
  learned initial guess, for gradient checks.

Parity status per function is listed in each module's header.
"""
