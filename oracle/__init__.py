"""Plain FP64 CPU oracle for the multilevel spatial BLUP solve.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP library.

Every function follows the paper (Castrillon-Candas, "Spatial best linear
unbiased prediction: a computational mathematics approach for high
dimensional massive datasets", arXiv:1701.00285) and cites the section,
equation or algorithm it restates:

  matern   Matern covariance (Definition in Sec. 3.1 and the half-integer
           remark after it), its rho-derivative, dense covariance blocks
  design   total-degree monomial design matrix X (Sec. 2, TD index set)
  kdtree   kd-tree with the max-variance / median split (Algorithms
           "Rule", "InitialTree", "MakeTree", Sec. 3.1)
  basis    multilevel basis W, L by per-cell SVD (Sec. 3.1 construction)
  blup     classic GLS / kriging (eqs. GLSbeta, KrigBLUP), the multilevel
           predictor (Sec. 5.2, eqs. Spatial:eqn1-3), quadratic form and its
           log-rho gradient
  brute    brute-force covariance sums (math.fsum double loop, row blocks)

Parity status of each function is listed in its module docstring; every
function here is pinned by a CPU test in tests/ against something other
than itself (a library routine, a closed form, an invariant, the paper's
printed numbers, or brute force).
"""
