"""Plain FP64 CPU oracle of the Fourier-Galerkin chemo-mechanical hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import or run anything in this package.
The product path (the HIP library and its Python binding) never calls it and
shares no code with it.

The oracle is deliberately slow and literal: numpy / scipy in float64, the
method's steps in the paper's order and notation, library FFTs / dense
linear algebra as the only primitives.  Citations name the section, equation
(number and LaTeX label) or algorithm of Zarzoso, Roque, Montero-Chacon,
Segurado, "An FFT based chemo-mechanical framework with fracture"
(arXiv:2411.16583).

Modules
-------
spectral      frequencies, rotated-scheme vector, projection G, 7-point symbol
constitutive  compressible Neo-Hookean P and K with swelling and degradation
krylov        CG / PCG (Hestenes-Stiefel)
mechanics     Newton-CG equilibrium (Alg. 1), residual err_res (eq. 31)
fracture      driving force D_f, history H, phase-field PCG (Alg. 2)
chemistry     chemical potential, mobility, Fick backward-Euler Newton (Alg. 3)
staggered     global staggered scheme (Alg. 4)
adjoint       adjoint sensitivity of <P_11> to log E and Omega
dense         dense real-space operators for brute force on tiny grids
laminate      exact laminate solution

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(tests/test_oracle_*.py) against closed forms, invariants, brute force or
library routines, except where its docstring says "parity unpinned".
"""
