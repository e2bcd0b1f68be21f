"""Plain, slow, FP64 CPU oracle of the multigrid ensemble Kalman filter (MEnKF).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and
the bench's CPU-baseline leg use it.  It shares no code with the HIP
library; the only common dependency is the ``synthetic`` input generator,
which holds none of the method's arithmetic.

Every function follows a passage of Moldovan, Lehnasch, Cordier & Meldi,
"A multigrid/ensemble Kalman filter strategy for assimilation of unsteady
flows" (J. Comput. Phys., arXiv 2012.10091), cited by section, equation or
algorithm.  Where the paper is silent the reading taken is stated in the
docstring.  NumPy/SciPy FP64 throughout; LAPACK Cholesky and triangular
solves are the only library linear algebra.

Modules
  grids     projection operators Pi_C and Pi_F (Sec. 2.2)
  models    Burgers and 2D compressible Navier-Stokes discretisations and
            explicit time advance (Sec. 2.2, eqs. of Secs. 4 and 6)
  obs       observation operators H^F and H^C (eq. of the observation model)
  rng       Philox4x32-10 counter generator and Box-Muller normals
  enkf      stochastic EnKF analysis with anomaly matrices (Algo. 1 / Algo. 3)
  kf        closed-form Kalman filter gain (Sec. 2.1.1) - pin only
  smooth    relaxed matrix-splitting (Jacobi) iteration on the fine grid
  cycle     one MEnKF assimilation cycle (Algo. 4)
  diag      relative RMSE and conservativity residual Gamma
  net       learned convolutional prolongation, forward and backward
"""
