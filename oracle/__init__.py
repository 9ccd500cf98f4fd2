"""CPU oracle for the k-blocked LR-CCSD sigma path (test infrastructure).

This package is test infrastructure only.  It is a plain, slow, fp64
implementation of what the paper's linear-response CCSD method computes,
written from the paper's equations (Sec. II.B: Eqs. ene, t1, t2, D, rhs,
tx1, tx2, lrf) and the textbook spin-orbital CCSD they follow.  Only the
test-suite, the smoke entry point and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the HIP library.

Normalisation: the oracle works in "crystal" normalisation on collective
indices P = (p, k_p) (Sec. II.A, Table index): a plain molecular spin-orbital
CCSD on N_O = Nk*o occupied and N_V = Nk*v virtual orbitals whose two-electron
integrals are v = v'/Nk, with v' the per-cell integrals built from the
Cholesky vectors.  The paper writes every two-electron quantity scaled by
Nk (each free k-sum carries 1/Nk); `layout` converts between the two.

Modules
  layout     k-block <-> dense collective conversions, dense integrals
  ccsd       CCSD residual Omega(T; f, v) and energy E(T; f, v)
  solvers    CCSD ground state (Jacobi + DIIS) and a GMRES linear solver
  response   sigma = A X (exact 5-point stencil), xi, lambda, eta, F, alpha
  fockspace  determinant-space brute force (pins the above)
"""
