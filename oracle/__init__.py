"""CPU FP64 oracle for the retrieved method-of-moments system (TEST INFRASTRUCTURE).

This package is test infrastructure only.  Nothing in the GPU library imports,
links or executes it; only the tests, the smoke check and the CPU-baseline leg
of the benchmark may call it.  It shares no code with the GPU path: the only
common inputs are the seeded geometry/codebook arrays of the ``workloads``
package, which contains no electromagnetic arithmetic.

What it computes (arXiv 2112.05082):
  * the Galerkin EFIE matrix Z I = U of eq. (1) on RWG bases (Sec. II-A),
    evaluated *directly on the active patches* of a codebook, which is the
    explicit retrieval Z_k = Z(active, active) of Sec. III-A;
  * the macro-unit displacement blocks Z(d) and the implicit retrieval of
    eqs. (3)-(6) as a plain block-Toeplitz product (``retrieval``);
  * plane-wave excitation, radiation vectors, RCS, dense LU and GMRES,
    and fully pivoted ACA of far blocks.

Every function is FP64 / complex128 and favours clarity over speed.

Parity pins: each module's functions are checked in tests/test_oracle_*.py
against quadrature exactness, polar-coordinate numerical integration,
reciprocity, a discrete power-balance identity, a closed-form excitation,
mirror symmetry, mesh-refinement convergence and the physical-optics limit of
a large plate.  The RCS against physical truth for the paper's own unit cells
is parity unpinned: the paper prints no RCS values.
"""
