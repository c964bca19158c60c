"""CPU oracle for the FIFA-GP hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 NumPy/SciPy code written from the paper (Moran & Wheeler,
"Fast increased fidelity approximate Gibbs samplers for Bayesian Gaussian process
regression", arXiv 2006.06537).  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It shares
no code with the HIP library: the only common module is ``workloads`` (seeded input
draws, no arithmetic of the method).

Modules
  rng     -- Philox4x64-10 counter generator, Box-Muller normals, Marsaglia-Tsang Gamma
  kernels -- covariance kernels k_1 (unit amplitude) of Sections 2.1 and 4.1
  dense   -- O1: exact dense GP (Eqs. 2-7), Lemma/Theorem quantities, KL divergence
  hodlr   -- O2: canonical HODLR build / symmetric factor / solve / log-det (Section 3,
             Algorithm 1 requirements, SI "HODLR decomposition and factorization")
  sampler -- Algorithm 1, Algorithm 1.h and the Gibbs sweep f -> tau -> sigma_f^-2 -> rho
  kalman  -- O(n) state-space recursion for the exponential kernel (exact large-n pin)
"""
