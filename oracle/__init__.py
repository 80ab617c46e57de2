"""FP64 CPU oracle for the statically condensed spectral-element Helmholtz operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle computes the plain definitions of Huismann, Stiller & Froehlich,
"Factorizing the factorization" (arXiv 1601.08179), slowly and explicitly:

* 1D GLL basis, diagonal (GLL-lumped) mass matrix M, stiffness matrix K
  (Sec. 3, the 1D mass/stiffness definitions and the GLL paragraph);
* the element Helmholtz operator as an explicit sum of Kronecker products
  (Sec. 3, eq. "helmholtz_operator", metric coefficients eq. "metriccoeffelement");
* the statically condensed element operator H_BB - H_BI H_II^-1 H_IB and the
  condensed right-hand side (Sec. 4, eq. "condensation_system"), via a dense
  Cholesky factorisation of H_II -- no fast diagonalisation;
* explicit global numbering and gather/scatter R, R^T (Sec. 3, the discrete
  system R H_L R^T u_G = R F_L);
* direct solves of the condensed and of the full uncondensed system, interior
  recovery (Sec. 4, Algorithm 1), a block-Jacobi PCG in the physical basis (the
  "BC" solver of Sec. 8), and adjoint gradients.

Conventions (fixed once, used everywhere):
* element arrays are indexed u[k][j][i] with i (direction x1) fastest; a
  Kronecker product A (x) B (x) C acts with C on i, B on j and A on k (this is
  forced by the metric coefficient d_1 = J*4/h_1^2 multiplying M (x) M (x) K);
* the global GLL node (I1, I2, I3) has lexicographic number
  I1 + (n1*p+1)*(I2 + (n2*p+1)*I3).

Every function cites the passage of the paper it follows.  The functions take
plain numpy arrays; seeded inputs come from the separate ``workloads`` module,
which holds none of the method's arithmetic.
"""

# submodules: gll, element, mesh, operators, grads (import them explicitly)
