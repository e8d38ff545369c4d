"""Pins of the oracle's multiple-relaxation-time collision for the pressure
lattice (D2Q9; the paper says its BGK model extends to MRT, Section 3).

  * the moment basis is orthogonal with the row norms of the D2Q9 basis and
    the pressure equilibrium has no flux or stress moments and no mass;
  * with every rate equal to 1/tau_f the collision is BGK (to rounding),
    walls and a source included;
  * with rho, e and epsilon relaxed at one rate the rest population does not
    reach the moving ones (the GPU does not store it);
  * with rates far from BGK the steady pressure and the velocity of eq. 3-10
    of a manufactured periodic Poisson problem converge at second order.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import lattice as lat_mod


def test_basis_orthogonal_and_equilibrium_moments():
    M = lat_mod.d2q9_moment_basis()
    G = M @ M.T
    assert np.array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    lat = lat_mod.d2q9()
    P = 0.731
    feq = np.array([(lat.w[0] - 1.0) * P] + [lat.w[i] * P for i in range(1, 9)])
    m = M @ feq
    assert abs(m[0]) < 1e-15                      # sum f^eq = 0 (eq. 3-3)
    assert np.abs(m[3:]).max() < 1e-15            # no flux, energy flux or stress


def _solver(collision, bc, Fp=None, tau_uniform=True, n=(12, 10)):
    nx, ny = n
    o = oracle.Solver("D2Q9", n, beta=0.3, Ds=0.05, coef=oracle.QuadraticKr(1.0, 4.0), bc_f=bc[0], bc_g=bc[1],
                      collision=collision)
    rng = np.random.default_rng(5)
    fshape = (1, ny, nx)
    K = np.ones(fshape) if tau_uniform else np.exp(0.4 * rng.standard_normal(fshape))
    o.set_fields(K, rng.uniform(0.2, 0.4, fshape), Fp=Fp)
    x = (np.arange(nx) + 0.5) / nx
    o.set_state(np.broadcast_to(1.0 - x, fshape) + 0.02 * rng.standard_normal(fshape),
                np.full(fshape, 0.4) if tau_uniform else rng.uniform(0.3, 0.6, fshape))
    o.update_coefficients()
    return o


WALLS = ([("abb", 1.0), ("abb", 0.0), ("bb",), ("abb", 0.5)], [("abb", 1.0), ("outflow",), ("bb",), ("bb",)])


def test_equal_rates_are_bgk():
    ref = _solver(None, WALLS)
    s = 1.0 / float(ref.tau_f.flat[0])
    assert np.ptp(ref.tau_f) <= 1e-15
    got = _solver(("mrt", s, s, s), WALLS)
    for _ in range(25):
        ref.f_iteration()
        got.f_iteration()
    assert np.abs(ref.f - got.f).max() <= 1e-14
    ref.saturation_step()
    got.saturation_step()
    assert np.abs(ref.g - got.g).max() <= 1e-14


def test_rest_population_decoupled():
    a = _solver(("mrt", 1.3, 1.1, 0.7), WALLS, tau_uniform=False)
    b = _solver(("mrt", 1.3, 1.1, 0.7), WALLS, tau_uniform=False)
    b.f[0] += np.random.default_rng(1).standard_normal(b.f[0].shape)
    for _ in range(10):
        a.f_iteration()
        b.f_iteration()
    assert np.abs(a.f[1:] - b.f[1:]).max() <= 1e-14
    # with e relaxed at another rate than rho the rest population leaks in
    M, Minv, _ = a.mrt
    neq = np.zeros(9)
    neq[0] = 1.0
    S = np.diag([1.3, 1.6, 1.3, 1.0, 1.1, 1.0, 1.1, 0.7, 0.7])
    assert np.abs((Minv @ S @ M @ neq)[1:]).max() > 1e-3


def _manufactured_errors(N, collision):
    """Steady pressure of -div(D_p grad P) = F_p on a periodic N x N box with
    P_e = A sin(kx) sin(ky), uniform D_p (S uniform), tau_f = 0.8."""
    L, A = float(N), 0.05
    k = 2 * math.pi / L
    cs2 = 1.0 / 3.0
    mu_n = 1.0
    # S = 0: D_p = K / mu_n; K chosen so tau_f = 0.8
    K = (0.8 - 0.5) * cs2 * mu_n
    bc = ([("periodic",)] * 4, [("periodic",)] * 4)
    o = oracle.Solver("D2Q9", (N, N), beta=0.3, Ds=0.05, coef=oracle.QuadraticKr(1.0, mu_n), bc_f=bc[0], bc_g=bc[1],
                      collision=collision, m=1)
    x = np.arange(N) + 0.0
    X, Y = np.meshgrid(x, x)
    Pe = A * np.sin(k * X) * np.sin(k * Y)
    Fp = 2 * k * k * (K / mu_n) * Pe
    o.set_fields(np.full((1, N, N), K), np.full((1, N, N), 0.3), Fp=Fp[None])
    o.set_state(np.zeros((1, N, N)), np.zeros((1, N, N)))
    o.update_coefficients()
    k_, r, st = o.pressure_solve(1e-13, 400000)
    assert st == oracle.OK
    P = o.pressure()[0]
    eP = np.sqrt(np.mean(((P - P.mean()) - Pe) ** 2)) / np.sqrt(np.mean(Pe ** 2))
    u = o.velocity()[:2, 0]
    ue = -(K / mu_n) * A * k * np.stack([np.cos(k * X) * np.sin(k * Y), np.sin(k * X) * np.cos(k * Y)])
    eu = np.sqrt(np.mean((u - ue) ** 2)) / np.sqrt(np.mean(ue ** 2))
    return eP, eu


@pytest.mark.parametrize("collision", [None, ("mrt", 1.4, 1.7, 0.6)])
def test_manufactured_poisson_second_order(collision):
    e16 = _manufactured_errors(16, collision)
    e32 = _manufactured_errors(32, collision)
    print(collision, e16, e32)
    for a, b in zip(e16, e32):
        assert a < 0.1
        assert 3.3 < a / b < 4.8, (a, b)
