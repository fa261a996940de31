"""Oracle: a plain, slow FP64 CPU implementation of the gradient-enhanced
damage hot path, written from the paper.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
(the HIP library and its Python binding) never does, and shares no code with
it.  The only module both sides use is the seeded input generator
(`workloads`), which holds none of the method's arithmetic.

Design: every quantity is built from its definition in plain PyTorch CPU
float64 operations.  Stresses, nonlocal conjugates and consistent tangents are
derivatives of the scalar free energy taken by automatic differentiation
(the paper's own route: only the energy is written by hand), the local
history update is solved by bisection on a bracket on which the yield
residual is monotone, global systems are solved with a direct sparse LU
(as the paper does with PETSc), and the adjoint gradient is the discrete
adjoint assembled from autograd vector-Jacobian products.

Modules
  icnn          input-convex network, effective weights  (ICNN, Sec. 4.2)
  constitutive  invariants, energy, yield, local update, qp response
  fem           shape functions, quadrature, element residual/tangent, CSR
  solve         Newton load path, direct solves, load-path loss adjoint

Every function names the passage of the paper it follows.  Readings where the
paper is silent are stated next to the code that takes them.
"""
