"""Plain, slow FP64 CPU oracle for the fast random-walk Kalman filter.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library; both sides read
the seeded inputs of the ``workloads`` module and nothing else.

Every function computes the plain definition of a quantity from the paper
(Saibaba, Miller, Kitanidis, "Fast Kalman filter using hierarchical matrices
and a low-rank perturbative approach"):

* ``kernels``   Matern covariance entries (Section 2.2.1, eq. maternfamily).
* ``rays``      straight-ray travel-time operator (Section 4.1, eq.
                lineartomography).
* ``direct``    y = Gamma x and Gamma H^T by direct O(N^2) kernel sums
                (never an H-matrix).
* ``kalman``    the standard Kalman filter with F = I (Algorithm 1 with the
                random-walk assumption of Section 2.1) and the exact
                cross-covariance recursion for constant H.
* ``gep``       the generalized eigenproblem H^T R^-1 H x = lambda Gamma^-1 x
                (Section 2.2.2, eqs. ghep and geneigendecomposition) and the
                closed-form per-mode recursion it implies for constant H
                (Section 2.3, Algorithm 3).
* ``ekf``       the extended Kalman filter for the Box-Cox observation model
                (the numerical experiments' extended filter, Algorithm 4,
                transform of eq. nonlinear).
* ``sampling``  conditional realizations s = s_hat + L s_u with L L^T = Sigma
                (Section 3.3).
"""
