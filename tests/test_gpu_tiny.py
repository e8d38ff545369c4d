"""Degenerate cases of the method on the GPU against the float64 oracle.

* The smallest grids: walled axes of three nodes (the least the one-sided
  differences of the initial gradients need; both sides refuse fewer) and
  periodic axes of one or two nodes beside walled ones, where a node is its
  own or its only neighbour across the periodic faces, on each lattice; a
  blocked launch's region then holds a single column or row of the domain.
* No flow: equal wall pressures on a uniform pressure and saturation.  The
  pressure populations sit at equilibrium (every deviation zero), so P stays
  the wall pressure, u is zero, and the saturation lattice only relaxes a
  uniform state that no flux moves.  On D2Q9 the moving populations of the
  equilibrium of eq. 3-4 depend on phi, so a phi that varies from node to
  node moves S by a truncation error even at rest (the D2Q5 / D3Q7
  equilibrium of Remark V does not depend on phi); the D2Q9 case takes a
  uniform phi.

Replays run the oracle's iteration counts, as in the other parity tests.
"""
import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, gpu_solver, oracle_solver, rel_l2, smooth_state
from tests.test_gpu_parity import TOL, _check_fields, _np

pytestmark = pytest.mark.gpu

WALLED = "walled"
MIXED_2D = ([("periodic",), ("periodic",), ("abb", 0.7), ("abb", 0.2)],
            [("periodic",), ("periodic",), ("abb", 0.9), ("bb",)])
MIXED_3D = ([("periodic",), ("periodic",), ("abb", 0.7), ("abb", 0.2), ("bb",), ("abb", 0.5)],
            [("periodic",), ("periodic",), ("abb", 0.9), ("bb",), ("bb",), ("bb",)])
TINY = [("D2Q5", (3, 3), WALLED), ("D2Q5", (4, 3), WALLED), ("D2Q5", (3, 5), WALLED),
        ("D2Q5", (1, 5), MIXED_2D), ("D2Q5", (2, 3), MIXED_2D),
        ("D3Q7", (3, 3, 3), WALLED), ("D3Q7", (4, 3, 3), WALLED),
        ("D3Q7", (1, 3, 4), MIXED_3D), ("D3Q7", (2, 3, 3), MIXED_3D),
        ("D2Q9", (3, 3), WALLED), ("D2Q9", (4, 3), WALLED), ("D2Q9", (1, 4), MIXED_2D), ("D2Q9", (2, 3), MIXED_2D)]


def _params(lattice, shape, bcs=WALLED):
    p, _ = inputs.injection_problem(shape, 1.0, 4.0, 11, 12)
    if lattice == "D2Q9":
        p = dict(p, lattice="D2Q9", beta=0.2)      # inside [max(phi)/2, 2 min(phi)] (eq. 3-4)
    if bcs != WALLED:
        p["bc_f"], p["bc_g"] = bcs
    assert p["lattice"] == lattice
    return p


@pytest.mark.parametrize("lattice,shape,bcs", TINY)
def test_tiny_grids_replay(lattice, shape, bcs):
    params = _params(lattice, shape, bcs)
    nx, ny, nz = params["shape"]
    fshape = (nz, ny, nx)
    seed = 3 + nx + 7 * ny + 31 * nz
    K = f32(5 / 6 * np.exp(inputs.gaussian_random_field(fshape if nz > 1 else (ny, nx), 4.0, seed))
            .reshape(fshape))
    phi = f32(inputs.uniform_field(fshape, 0.15, 0.3, seed + 1))
    P0, S0 = (f32(a) for a in smooth_state(fshape, seed + 2))
    periodic = False            # every case has a walled axis: P is not defined up to a constant
    print(f"tiny grid {lattice} {shape}", flush=True)
    o = oracle_solver(params, m=64)
    o.set_fields(K, phi)
    o.set_state(P0, S0)
    g = gpu_solver(params, m=64)
    g.set_fields(K, phi)
    g.set_state(P0, S0)
    for n, iters in enumerate([1, 10, 100]):
        o.update_coefficients()
        g.update_coefficients()
        k_o, _, _ = o.pressure_solve(-1.0, iters)
        k_g, _, _ = g.pressure_solve(-1.0, iters)
        assert k_o == k_g == iters
        _check_fields(o, g, f"{lattice} {shape} step {n} after {iters} iterations", periodic=periodic)
        o.saturation_step()
        g.saturation_step()
    _check_fields(o, g, f"{lattice} {shape} after three coupled steps", periodic=periodic)
    fg, gg = g.populations()
    assert rel_l2(o.f[1:], _np(fg)) <= TOL
    assert rel_l2(o.g, _np(gg)) <= TOL


@pytest.mark.parametrize("lattice,shape", [("D2Q5", (40, 24)), ("D3Q7", (20, 12, 9)), ("D2Q9", (40, 24))])
def test_no_flow_stays_at_rest(lattice, shape):
    params = _params(lattice, shape)
    nfaces = 6 if lattice == "D3Q7" else 4
    params["bc_f"] = [("abb", 0.5), ("abb", 0.5)] + [("bb",)] * (nfaces - 2)
    params["bc_g"] = [("abb", 0.3), ("outflow",)] + [("bb",)] * (nfaces - 2)
    nx, ny, nz = params["shape"]
    fshape = (nz, ny, nx)
    K = f32(5 / 6 * np.exp(inputs.gaussian_random_field(fshape if nz > 1 else (ny, nx), 4.0, 5))
            .reshape(fshape))
    phi = np.full(fshape, 0.25) if lattice == "D2Q9" else f32(inputs.uniform_field(fshape, 0.15, 0.3, 6))
    P0, S0 = np.full(fshape, 0.5), np.full(fshape, 0.3)
    print(f"no flow {lattice} {shape}", flush=True)
    o = oracle_solver(params, m=64)
    o.set_fields(K, phi)
    o.set_state(P0, S0)
    g = gpu_solver(params, m=64)
    g.set_fields(K, phi)
    g.set_state(P0, S0)
    for iters in (1, 70, 130):
        for s in (o, g):
            s.update_coefficients()
            s.pressure_solve(-1.0, iters)
            s.saturation_step()
    P, u, S = _np(g.pressure()), _np(g.velocity()), _np(g.saturation())
    # u is zero on both sides (to rounding in the oracle), so it is bounded
    # absolutely; P and S are compared with the oracle as everywhere else
    assert rel_l2(o.pressure(), P) <= TOL and rel_l2(o.saturation(), S) <= TOL
    assert np.abs(P - 0.5).max() <= 1e-7, np.abs(P - 0.5).max()
    assert np.abs(u).max() <= 1e-9, np.abs(u).max()
    assert np.abs(S - 0.3).max() <= 1e-6, np.abs(S - 0.3).max()
    assert np.abs(o.velocity()).max() <= 1e-12
