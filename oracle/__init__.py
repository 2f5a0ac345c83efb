"""Plain FP64 CPU oracle for the single-layer dual-mesh BEM (test infrastructure only).

This package is the checker, not the product.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the GPU library
never calls into it and shares no code with it.

Everything here is written from the paper's definitions (Sec. II: eqs. for the
operators L^(A), L^(phi), K~, the discretised internal, equivalent and external
AEFIE and the final system) in float64/complex128, with numpy/scipy as the only
numerical primitives (LAPACK LU for the dense solves).  Where the paper defers a
definition to a reference that is not reproduced (RWG normalisation, the charge
neutrality maps F and B, Buffa-Christiansen functions, quadrature), the module
that implements it states the reading it takes.

Modules
  constants   physical constants and material wavenumbers (eq. epsrc, Sec. II-B)
  mesh        topology, RWG data, incidence D, charge maps F/B, barycentric
              refinement and Buffa-Christiansen coefficients
  quadrature  triangle rules (Radon 7-point, 3-point), Gauss-Legendre, Duffy
  potentials  closed-form static integrals over a flat triangle
  operators   Galerkin fill of L^A, L^phi, K~, the Gram matrix I_x and the
              plane-wave right-hand side
  systems     augmented, reduced and final (explicit-Y) systems, LU solves,
              far-field / RCS of the differential current
  mie         Mie series for a homogeneous dielectric sphere (far-field amplitudes and
              the scattered near field)
  nearfield   E and H at exterior points radiated by the differential current and
              charge (mixed potentials, singularity extraction near the surface)
  brute       whole Galerkin entries of L^A, L^phi, K~ by brute force (singularity-
              cancelling maps of each triangle pair onto the 4-cube, tensor
              Gauss-Legendre): no extraction, no closed forms, no rule set Q; it pins
              the near-pair fill of `operators`
"""
