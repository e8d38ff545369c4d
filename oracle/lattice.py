"""Discrete-velocity lattices of the double-distribution LB model.

TEST INFRASTRUCTURE: part of the CPU oracle (see oracle/__init__.py).

D2Q9 follows the paper exactly (Section 3, eq. (3-5), (3-5a), (3-6), (3-6a)).
D2Q5 and D3Q7 are the DnQ(2n+1) lattices of Remark V (eq. (3-4b)); the paper
gives their equilibrium but not their weights, so the weights here are a
reading: the weights must give sum w = 1, sum w c = 0 and
sum w c c = c_s^2 I (the moment conditions eq. (3-7)), which for an
axis-aligned lattice means c_s^2 = 2 w_1 c^2.  The choices are
  D2Q5: w_0 = 1/3, w_{1..4} = 1/6, c_s^2 = c^2/3;
  D3Q7: w_0 = 1/4, w_{1..6} = 1/8, c_s^2 = c^2/4.
The source weights wbar follow the pattern of eq. (3-5a): wbar_0 = 0 and the
moving directions share the source equally, wbar_{i>=1} = 1/(Q-1).

Velocity ordering: index 0 is the rest velocity; 1..4 of D2Q5 and D2Q9 point
at angles 0, 90, 180, 270 degrees as in eq. (3-6); D2Q9 5..8 are the
diagonals at 45, 135, 225, 315 degrees; D3Q7 is D2Q5's ordering followed by
+z, -z.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Lattice:
    name: str
    dim: int
    e: np.ndarray        # (Q, 3) integer unit vectors; c_i = c * e_i
    w: np.ndarray        # (Q,) equilibrium weights omega_i
    wbar: np.ndarray     # (Q,) source weights bar-omega_i
    cs2_c2: float        # c_s^2 / c^2
    opp: np.ndarray      # (Q,) index of the opposite velocity

    @property
    def Q(self):
        return self.e.shape[0]

    @property
    def odd(self):
        """True for the DnQ(2n+1) family, which uses the eq. (3-4b) equilibrium."""
        return self.name in ("D2Q5", "D3Q7")


def _opposites(e):
    opp = np.empty(len(e), dtype=np.int64)
    for i, ei in enumerate(e):
        (j,) = [j for j, ej in enumerate(e) if np.array_equal(ej, -ei)]
        opp[i] = j
    return opp


def _make(name, dim, e, w, cs2_c2):
    e = np.asarray(e, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    q = len(e)
    wbar = np.full(q, 1.0 / (q - 1))
    wbar[0] = 0.0
    return Lattice(name, dim, e, w, wbar, cs2_c2, _opposites(e))


def d2q9():
    # eq. (3-6): i = 1..4 at (i-1) pi/2, i = 5..8 at (2i-9) pi/4 with length sqrt(2)
    e = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
         (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4          # eq. (3-5)
    return _make("D2Q9", 2, e, w, 1.0 / 3.0)            # eq. (3-6a)


def d2q5():
    e = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0)]
    w = [1 / 3] + [1 / 6] * 4
    return _make("D2Q5", 2, e, w, 1.0 / 3.0)


def d3q7():
    e = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    w = [1 / 4] + [1 / 8] * 6
    return _make("D3Q7", 3, e, w, 1.0 / 4.0)


def get(name):
    return {"D2Q9": d2q9, "D2Q5": d2q5, "D3Q7": d3q7}[name]()


def d2q9_moment_basis():
    """Moment basis of the D2Q9 multiple-relaxation-time collision (the
    orthogonal basis of Lallemand and Luo, Phys. Rev. E 61 (2000) 6546, which
    the paper cites for MRT), rows in the order
        rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy
    built from the velocities e_i of d2q9() (|e|^2 = e_x^2 + e_y^2):
        1, -4 + 3|e|^2, 4 - 21/2 |e|^2 + 9/2 |e|^4, e_x, (-5 + 3|e|^2) e_x,
        e_y, (-5 + 3|e|^2) e_y, e_x^2 - e_y^2, e_x e_y.
    Returns a (9, 9) float array M with m = M f."""
    e = d2q9().e.astype(np.float64)
    ex, ey = e[:, 0], e[:, 1]
    c2 = ex * ex + ey * ey
    rows = [np.ones(9), -4.0 + 3.0 * c2, 4.0 - 10.5 * c2 + 4.5 * c2 * c2, ex, (-5.0 + 3.0 * c2) * ex,
            ey, (-5.0 + 3.0 * c2) * ey, ex * ex - ey * ey, ex * ey]
    return np.stack(rows)
