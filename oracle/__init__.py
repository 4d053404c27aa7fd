"""Oracle: a plain, slow FP64 CPU implementation of the coupled phase-field LBM step.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  The product library (the HIP
kernels behind the C ABI and their Python binding) never calls into it, and
the oracle shares no code, tables or helpers with that library.

Contents
  lattice   velocity sets (D3Q15, D3Q27, D2Q9), weights, Gram-Schmidt moment
            matrices (eq. mrt)
  pflbm     one time step, S1-S17, written from the paper's equations
  adjoint   reverse-mode gradients of the oracle by torch autograd
  analytic  closed forms (capillary/gravity waves, Poiseuille, Laplace)

Pinned by tests/test_oracle_*.py against closed forms, invariants and
special cases.  Parity unpinned (definitional choices with no external
check beyond oracle == GPU): the explicit u' inside the viscous force, the
synchronous time levels of the two sub-steps, the equilibrium initialisation
details and the default high-order rate s_high = 1.
"""
from .lattice import CS2, D2Q9, D3Q15, D3Q27  # noqa: F401
from .pflbm import (Grid, OracleParams, amplitude, collide, init_equilibrium,  # noqa: F401
                    interface_crossing, moments, reductions, run, step, stream)
