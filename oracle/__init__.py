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
  * the tau_f = 1 fixed point with walls equals a direct sparse solve of the
    matching finite-difference system;
  * a layered medium (tau_f from about 0.5 to 50 along x, D2Q5 and D3Q7):
    the fixed point is the series-resistance closed form and the local
    velocity is the constant flux, to rounding;
  * the initial non-equilibrium parts have the moments of Appendices A and B;
  * collision invariants and the exact mass ledger;
  * Example 1 of Section 4: the printed error bound and second order;
  * Example 2: the printed bound for P and u; second order of S at fixed
    tau_g (Fig. 10); errors falling with beta at phi = 0.5 (Fig. 11); the
    saturation error at fixed c is the modified-equation term of eq. (3-2)
    (its size, its 1/c^2 scaling, and its removal by the compensating source);
  * second-order convergence of the manufactured problem on D2Q5 (P, u, S)
    and D3Q7 (P, u, S);
  * agreement with a finite-volume Darcy solve as the grid is refined.
"""
from . import lattice
from .lattice import Lattice, d2q5, d2q9, d3q7
from .solver import (FACES, NOT_CONVERGED, OK, UNSTABLE, GivenCoefficients,
                     QuadraticKr, Solver)

__all__ = ["lattice", "Lattice", "d2q5", "d2q9", "d3q7", "FACES", "OK",
           "NOT_CONVERGED", "UNSTABLE", "GivenCoefficients", "QuadraticKr",
           "Solver"]
