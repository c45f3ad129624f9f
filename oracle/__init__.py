"""FP64 CPU oracle for the line-periodic FBC boundary update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything under this package: only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code, table or constant
generator with the HIP library; both sides are fed from the separate seeded
input module ``fbc_workloads``.

Modules
-------
lattice    fcc basis, nearest-neighbour central springs, dynamical matrix D(q)
           (Section 2.2.1, linearised operator L_h; Appendix B, Fourier symbol of K_h)
supercell  brute-force stiffness of the periodic torus supercell and its
           pseudo-inverse / CG solve (Section 2.3.2, Green operator with G L_h = I)
green      line-mode Green blocks G^(m; dn1, dn2) by Brillouin-zone summation
           (Appendix B, inverse semi-discrete Fourier transform, discretised)
apply      rFFT -> per-mode complex matrix product -> irFFT; pad update and
           mean removal (Section 2.3.2, eq. flexbc.up=Gpipl*fipl and eq. mean(u^p)=0)
relax      residual-based relaxation (Section 2.3.3, eq. alpha, Algorithm 2) and
           the harmonic side of Algorithm 1
split      BF16 hi+lo split representation, emulated on the host
mlp        4-layer MLP forward / analytic backward in FP64
cgf        continuum (anisotropic) Green function in the line-mode representation
           (Section 3.1, eq. cgf; Appendix B)

Every function cites the passage it follows.  Pins (tests/test_oracle_*.py)
tie each function to something other than itself.
"""
