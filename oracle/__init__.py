"""Plain FP64 CPU oracle for the high-order DG S_N sweep inside the Second
Moment Method (Olivier & Haut, "High-Order Finite Element Second Moment
Methods for Linear Transport").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It is written from the paper's equations for readability, not for
speed, and shares no code with the HIP library.

Modules
  quadrature  level-symmetric S_N sets; Gauss-Legendre / Gauss-Lobatto rules
  fem         Q_p nodal basis, Q_m mesh map, element and face data (Sec. 3)
  transport   upwind DG sweep and angular moments / SMM closures (Sec. 4)
  smm         interior-penalty and continuous (CG) SMM moment systems and the
              fixed point (Sec. 2.3, 5.1)
  cnn         plain convolutional network forward/backward for the warm start

Functions whose result the tests cannot tie to the paper or to mathematics
say "parity unpinned" in their docstring.
"""
