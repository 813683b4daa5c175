"""Plain FP64 CPU oracle for the NysADMM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py use it.  It shares no code with the HIP library; both sides
receive the same seeded inputs from paper_2202_11599_amd.synth, which holds
none of the method's arithmetic.

Everything here is NumPy/SciPy in float64, written to be checked against the
paper (Zhao, Frangella, Udell: "NysADMM: faster composite convex optimization
via low-rank approximation", ICML 2022) by eye:

  nystrom   Algorithm RandNysAppx, eq. (NysAppx), eq. (Nyspreconditioner),
            Algorithm AdaptiveRandNysAppx, eq. (deff)
  pcg       Algorithm Nystrom PCG, the subproblem (ADMMSubProb) by a dense solve
  admm      Algorithm NysADMM / Inexact ADMM for lasso (eq. 2) and l1-logistic
            regression (eq. 9), the residuals of Section 2.1, KKT residual (31)
  mlp       the warm-start network (not in the paper), FP64 forward/backward/Adam
  svm       the kernel SVM dual (eq. 8) by NysADMM: RBF kernel, projection onto
            {0 <= z <= C, b^T z = 0}, duality gap
  rng       the Gaussian entries of the test matrix of Algorithm RandNysAppx
            when the library draws them: Philox4x32-10 and Box-Muller

Parity status of every function is stated in its module header.
"""
