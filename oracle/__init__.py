"""CPU oracle for temporal-GP inference in sparse-precision form.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
device path.

Modules
  ssm     state-space form of the covariance functions (paper Sec. 2.1,
          eq. ss_matern), built on scipy's matrix exponential
  dense   O(N^3) textbook GP (eq. ml2, mean2, k3 with a dense solve), float64
          and mpmath
  kalman  covariance-form Kalman filter + RTS smoother (the paper's KF
          comparison method, Sec. 4.2) with a tangent-linear gradient
  btd     sequential block-tridiagonal elimination of the posterior precision
          (Theorem 1, Sec. 3.1 subproblems 1-4: Thomas algorithm, determinant,
          Takahashi selected inverse, trace gradient of eq. dd1)
  native  ctypes front end of ``c/oracle.c``, the same sequential elimination
          in plain C for large N
"""
