"""Plain FP64 CPU oracle for the Leja phi_l(hJ)v action -- TEST INFRASTRUCTURE.

This package is the slow, obviously-correct reference the HIP library is
checked against.  It is test infrastructure only: nothing but the tests, the
smoke check and the bench's CPU-baseline leg may import it, and the product
path never calls it (the HIP library fails loudly when it is not built instead
of falling back here).  It shares no code with the HIP library; both take their
inputs from the separate `workloads` package, which holds no method arithmetic.

Modules (each function cites the passage of the paper it follows):
  points      Leja points on [-2, 2]                       (Sec. 2.2)
  phi         scalar phi_l(z), high precision              (Sec. 1 definition)
  divdiff     Newton divided differences in FP64           (Sec. 2.2)
  splitmix    SplitMix64 counter-based generator (power-iteration start vector)
  operators   periodic 2nd-order stencils f(u), J(u)v      (Sec. 3, Sec. 4)
  power       power-iteration spectral bound               (Sec. 2.2, Sec. 5.1)
  leja        interval map, Newton recurrence, stop/reject, vertical form,
              substepping                                   (Sec. 2.1, 2.2, 4)
  integrators EXPRB2, EXPRB43, EPIRK4s3 stage driver        (Sec. 1, eqs. of Sec. 5.1, 5.4)
  exact       closed forms used as pins: elementwise phi for diagonal J,
              Fourier diagonalisation, dense Pade expm of the augmented
              matrix (Sec. 2.1 theorem)
  mlp         FP64 forward/backward of the learned-proposal MLP
  features    state statistics fed to the learned proposal
"""
