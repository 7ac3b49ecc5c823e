"""Reference (oracle) implementation of the rational-function log-determinant
estimator of Colthurst, Vasudevan, Lottes and Patton, "Fast Approximate
Determinants Using Rational Functions" (arXiv 2405.03474).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64, CPU-only
restatement of what the method computes.  It exists to check the HIP library
and shares no code with it.  Only the test suite, the smoke check of the
graft entry point and the CPU-baseline leg of the benchmark may import it;
the product path never does.

Modules:
  rational  -- the Kelisky-Rivlin approximants r_k (eq. 1) and their
               partial-fraction form (Table 1)
  rng       -- the counter-based random stream used for probes and sketches
  gp        -- RBF / Matern-5/2 covariance matrices (Section 3 kernels)
  precond   -- randomized truncated-SVD preconditioner (Section 2, Appendix)
  estimate  -- the estimator output of Algorithm 1 with exact shifted solves,
               exact Cholesky log det, and the bias decomposition
  lanczos   -- Algorithm 1 as printed: t Lanczos steps per probe and the
               shifted tridiagonal solves
  gradient  -- d log det M / d(lengthscale, variance, noise) by Hutchinson over
               probe solves
  mlp       -- the surrogate network: forward, chain-rule gradient, Adam, features
"""
