"""CPU oracle for the adaptive multigrid solve of D(U) psi = chi.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
restatement of what the paper (Brannick, Brower, Clark, Osborn, Rebbi,
"Adaptive Multigrid Algorithm for Lattice QCD", arXiv:0707.4018) computes.
It exists to check the HIP path; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it.  It shares no code with the
HIP library and never imports it.

Modules:
  lattice  geometry, shifts and the gamma matrices
  dirac    the Wilson-Dirac operator D and D^dagger (definition after Eq. (1))
  mg       blocks, chirally split prolongator, Galerkin coarse operator
           (Eq. (2)), MR smoother (Eq. (4) read for D), V-cycle (five-step
           list before Eq. (3)), GCR/FGCR, CGNR, adaptive setup (text around
           Eq. (5))
  spectrum critical-mass estimate from the spectrum of D
  cnn      reference forward/backward of the null-vector proposal network
"""
