"""CPU oracle for the double-distribution lattice Boltzmann model of
Chai, Liang, Du and Shi, "A lattice Boltzmann model for two-phase flow in
porous media" (arXiv:1808.07554).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, float64 NumPy
implementation written from the paper's equations, used to check the HIP
path.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it; the product path never does.  It shares no code with the HIP
library (the two see the same seeded inputs and nothing else).

Pins (each checked by a test that needs no GPU):
  * lattice tables and the moment conditions of eq. (3-7): exact identities;
  * tau_f = 1 on D2Q5/D3Q7 reduces the pressure iteration to textbook Jacobi
    on the 5/7-point Laplacian, and its local gradient to central differences;
  * tau_g = 1 on D2Q5 reduces the saturation step to forward-time
    central-space differencing;
  * the fixed point of the pressure iteration equals a dense linear solve of
    the affine sweep on tiny grids (any heterogeneous tau_f);
  * collision invariants and the exact mass ledger;
  * Examples 1 and 2 of Section 4 (D2Q9): the printed error bounds and
    second-order convergence;
  * second-order convergence of the D2Q5 manufactured problem;
  * agreement with a finite-volume Darcy solve as the grid is refined.
"""
from . import lattice
from .lattice import Lattice, d2q5, d2q9, d3q7
from .solver import (FACES, NOT_CONVERGED, OK, UNSTABLE, GivenCoefficients,
                     QuadraticKr, Solver)

__all__ = ["lattice", "Lattice", "d2q5", "d2q9", "d3q7", "FACES", "OK",
           "NOT_CONVERGED", "UNSTABLE", "GivenCoefficients", "QuadraticKr",
           "Solver"]
