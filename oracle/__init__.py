"""FP64 CPU oracle for adaptive-multigrid Wilson-clover solves (TEST INFRASTRUCTURE).

This package is a plain, slow, deliberately unoptimised restatement of what
the method computes (Clark et al., "Accelerating Lattice QCD Multigrid on
GPUs Using Fine-Grained Parallelization", arXiv:1612.07873): the
Wilson-clover matrix of Eq. (2), the adaptive setup of Sec. 3.4 (null
vectors, blockwise QR, Galerkin product), the coarse operator of Eq. (3),
the transfer operators of Sec. 6.6 and the K-cycle GCR solver of Sec. 7.1.

It is test infrastructure only.  Nothing in the product library imports,
links or executes it; only the tests, the smoke check of the build entry
point and the CPU-baseline leg of the benchmark may call it.  It shares no
code with the HIP path; the only common module is ``synth`` (seeded random
inputs, no method arithmetic).

Everything is complex128.  Conventions (fixed here, and restated in the C
header of the library):
  * site index i = x0 + L0*(x1 + L1*(x2 + L2*x3)), dimension 3 is time;
  * fine fields [V][4][3] (spin, colour), dof index f = 3*spin + colour;
  * chirality chi(f) = f // (dof/2): spins {0,1} are chi=0, {2,3} chi=1;
  * coarse index n = chi*Nvec + k;
  * direction d = 2*mu + 0 (forward hop, acts on u(x+mu)) or + 1 (backward);
  * periodic space, antiperiodic time for the fine operator; the coarse
    operator wraps periodically (the sign already sits inside its links).
"""
