"""FP64 CPU oracle of the local spectral stage of MS-GFEM (test infrastructure).

This package is a plain, slow, deliberately unoptimised restatement of what
the method computes, used only to check the HIP library: by the tests, by the
smoke check and by the CPU-baseline leg of the benchmark.  Nothing in the
product path imports it.  It shares no code with the HIP path; the only common
module is the seeded input generator ``paper_2211_13893_amd.synth``.

Modules (each function cites the passage of the paper it follows):
  material  - orthotropic ply tensors and their rotation (Sec. 2, Sec. 5.1)
  fem       - Q1 hexahedral element stiffness, assembly, traction loads (Sec. 2)
  decomp    - subdomains, DoF classes B1/B2/B3, partition of unity (Sec. 3.1, 4.2, 4.3)
  gevp      - the A-harmonic local GEVP, Schur-reduced and augmented (Sec. 3.3, 4.3)
  coarse    - particular functions, coarse Galerkin problem, fine solve (Sec. 3.3, 4.4)
  geneo     - classic GenEO local GEVP and two-level PCG (Sec. 3.2, Sec. 5.3)
"""
