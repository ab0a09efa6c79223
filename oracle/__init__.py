"""Oracle for the compact finite-difference hot path.

TEST INFRASTRUCTURE ONLY: a plain, slow, independent CPU implementation of
what the GPU library computes, written from arXiv 2302.14858.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product library never does, and the two share no code.

* ``oracle.schemes``  - scheme construction (Taylor matching, spectral tuning,
  matched closures) in exact or high-precision arithmetic.
* ``oracle.lines``    - FP64 line operator: explicit RHS stencil, closure rows,
  banded elimination, cyclic (periodic) solve; plain C behind ctypes.
* ``oracle.wave``     - the first-order wave system under classical RK4: the
  closed-form evolution of one Fourier mode and a plain stepped integrator.
* ``oracle.iterate``  - hybrid iteration of the block closures.
* ``oracle.dissipation`` - Kreiss-Oliger dissipation by repeated differences.
* ``oracle.mixed``    - symmetrised mixed second derivatives 1/2 (D_i D_j + D_j D_i).
* ``oracle.biased``   - biased (upwind) schemes U, V, X with their xi-closures,
  their line operator (dense solve) and the upwind selection by a velocity
  field.

The dense assembled matrices of Eqs. diff_mat_subL/R and the embedded
operator of Eq. iter_scheme that pin ``oracle.lines`` are written out in the
tests themselves (``tests/test_oracle_lines.py``), with numpy.
"""
