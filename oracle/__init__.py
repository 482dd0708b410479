"""Plain FP64 CPU oracle for the 3-D Euler modal DG residual and its SSP-RK3 update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package;
it exists to check the HIP implementation.  It shares no code with it: its own
quadrature (SciPy Gauss-Jacobi roots), its own basis (exact symbolic expansion of
the PKD polynomials), its own geometry (face area vectors from cross products),
face-centric assembly (every unique face evaluated once and scattered to both
neighbours) and reverse-mode AD for the adjoint.

Parity pins: see the tests named test_oracle_*.py.  The paper (arXiv 2209.01877)
fixes the equations (Sec. II.A), the modal expansion (Sec. II.B, eq. 10), the weak
form with element, interior-face and boundary-face Gaussian integrals (eq. 11)
and the explicit RK time loop (Sec. III); basis, quadrature, flux (Rusanov) and
the RK variant (SSP-RK3) are the readings documented with each function.
"""
