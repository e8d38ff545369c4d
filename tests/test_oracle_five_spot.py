"""Pins of the oracle's per-link wall rules and of the five-spot problem
(Section 4.3) on the CPU.

  * a mixed face whose predicate selects every link (or none) is exactly the
    plain face rule;
  * the five-spot layout is symmetric under x <-> y, so P and S are (to
    rounding) after any number of steps; with a uniform D_p (S = 0, the
    first solve) the steady pressure is also odd about P = 1/2 under
    (x, y) -> (1 - x, 1 - y) (injector and producer exchange);
  * the steady pressure of the first solve approaches a finite-difference
    solution of the same mixed boundary value problem (a different
    discretisation, solved by a sparse direct solver) as the lattice is
    refined;
  * the binding's per-link condition lists select the same links as the
    oracle's midpoint predicate.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
from paper_1808_07554_amd import inputs
from tests.lbhelp import oracle_solver, smooth_state


def _mixed_problem(bc_f, bc_g, nx=8, ny=6):
    o = oracle.Solver("D2Q9", (nx, ny), beta=0.3, Ds=0.05, coef=oracle.QuadraticKr(1.0, 4.0),
                      bc_f=bc_f, bc_g=bc_g, m=1)
    fshape = (1, ny, nx)
    rng = np.random.default_rng(3)
    o.set_fields(np.exp(0.3 * rng.standard_normal(fshape)), rng.uniform(0.2, 0.4, fshape))
    P0, S0 = smooth_state(fshape, 11)
    o.set_state(P0, S0)
    for _ in range(3):
        o.update_coefficients()
        o.pressure_solve(-1.0, 7)
        o.saturation_step()
    return o


def test_mixed_face_with_uniform_predicate_is_the_plain_rule():
    yes = lambda x, y, z, t: np.ones_like(x, dtype=bool)
    no = lambda x, y, z, t: np.zeros_like(x, dtype=bool)
    plain_f = [("abb", 0.8), ("abb", 0.1), ("bb",), ("abb", 0.4)]
    plain_g = [("abb", 0.9), ("outflow",), ("bb",), ("abb", 0.2)]
    ref = _mixed_problem(plain_f, plain_g)
    mixed_f = [("links", yes, plain_f[0], ("bb",)), ("links", no, ("bb",), plain_f[1]),
               ("links", yes, ("bb",), ("abb", 0.3)), ("links", no, ("abb", 0.7), plain_f[3])]
    mixed_g = [("links", no, ("bb",), plain_g[0]), ("links", yes, plain_g[1], ("bb",)),
               ("links", no, ("abb", 0.5), ("bb",)), ("links", yes, plain_g[3], ("bb",))]
    got = _mixed_problem(mixed_f, mixed_g)
    assert np.array_equal(ref.f, got.f)
    assert np.array_equal(ref.g, got.g)
    assert ref.flux_ledger == got.flux_ledger


def _five_spot_oracle(N, m=1):
    p, fl = inputs.five_spot(N)
    o = oracle_solver(p, m=m)
    o.set_fields(fl["K"], fl["phi"])
    o.set_state(fl["P0"], fl["S0"])
    return o


def test_five_spot_symmetries():
    o = _five_spot_oracle(16)
    o.update_coefficients()
    assert np.ptp(o.Dp) == 0.0                 # S = 0 everywhere: uniform D_p
    k, r, st = o.pressure_solve(1e-13, 100000)
    assert st == oracle.OK
    P = o.pressure()[0]
    assert np.abs(P - P.T).max() <= 1e-14
    assert np.abs((P - 0.5) + (P[::-1, ::-1] - 0.5)).max() <= 1e-12
    # monotone fall from the injector to the producer along the diagonal
    assert np.all(np.diff(np.diag(P)) < 0)
    o.saturation_step()
    for _ in range(3):
        o.update_coefficients()
        o.pressure_solve(-1.0, 64)
        o.saturation_step()
    S, P = o.saturation()[0], o.pressure()[0]
    assert S.max() > 0.1                        # water has entered at the injector
    assert np.abs(S - S.T).max() <= 1e-14
    assert np.abs(P - P.T).max() <= 1e-14


def _fd_pressure(N, well=inputs.FIVE_SPOT_WELL, P_inj=1.0, P_prod=0.0):
    """Cell-centred five-point Laplace solve with the five-spot walls: a
    boundary face of a cell is Dirichlet (ghost value 2 P_w - P) where its
    midpoint lies in a well segment, no flux otherwise."""
    h = 1.0 / N
    c = (np.arange(N) + 0.5) * h
    rows, cols, vals = [], [], []
    b = np.zeros(N * N)
    for j in range(N):
        for i in range(N):
            r = j * N + i
            diag = 0.0
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < N and 0 <= jj < N:
                    rows.append(r)
                    cols.append(jj * N + ii)
                    vals.append(1.0)
                    diag -= 1.0
                    continue
                xm = 0.0 if ii < 0 else (1.0 if ii >= N else c[i])
                ym = 0.0 if jj < 0 else (1.0 if jj >= N else c[j])
                if xm < well and ym < well:
                    diag -= 2.0
                    b[r] -= 2.0 * P_inj
                elif xm > 1 - well and ym > 1 - well:
                    diag -= 2.0
                    b[r] -= 2.0 * P_prod
            rows.append(r)
            cols.append(r)
            vals.append(diag)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N * N, N * N))
    return spl.spsolve(A, b).reshape(N, N)


def test_five_spot_pressure_approaches_finite_differences():
    errs = []
    for N in (16, 32):
        o = _five_spot_oracle(N)
        o.update_coefficients()
        k, r, st = o.pressure_solve(1e-12, 200000)
        assert st == oracle.OK
        d = o.pressure()[0] - _fd_pressure(N)
        errs.append((np.abs(d).max(), np.abs(d).mean()))
    # the well ends are singular, so the agreement improves at below second order
    assert errs[0][0] < 0.02 and errs[1][0] < 0.7 * errs[0][0], errs
    assert errs[1][1] < 0.6 * errs[0][1], errs


@pytest.mark.parametrize("N", [12, 32])
def test_binding_link_lists_match_oracle_midpoints(N):
    from paper_1808_07554_amd import lbtp
    p, fl = inputs.five_spot(N)
    o = oracle_solver(p, m=1)
    lat = o.lat
    for lattice_rules in (p["bc_f"], p["bc_g"]):
        for face, rule in enumerate(lattice_rules):
            lists = lbtp.link_types(p["shape"], p["dx"], face, rule).reshape(N, 3)
            a, side = face // 2, face % 2
            for i in range(1, lat.Q):
                e = lat.e[i]
                if e[a] != (1 if side == 0 else -1):
                    continue          # not arriving through this face
                sl = [slice(None)] * 3
                sl[2 - a] = 0 if side == 0 else -1
                # the oracle's predicate on the cut links of population i: (z, along)
                along = np.broadcast_to(o._bvalue(rule[1], i, tuple(sl), 0.0), (1, N))[0]
                t = e[1 - a]
                slot = 0 if t == 0 else (1 if t < 0 else 2)
                want = np.where(along, lbtp._BC[rule[2][0]], lbtp._BC[rule[3][0]])
                assert np.array_equal(lists[:, slot], want), (face, i)
    if N == 32:          # each well segment: 4 normal links per face (1/8 of the side)
        lists = lbtp.link_types(p["shape"], p["dx"], 0, p["bc_f"][0]).reshape(N, 3)
        assert int(np.sum(lists[:, 0] == lbtp.BC_DIRICHLET)) == 4
