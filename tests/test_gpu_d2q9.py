"""D2Q9 (the paper's own lattice, eq. 3-4, 3-5, 3-6) on the GPU against the
float64 oracle, through the C ABI: replays of the oracle's iteration counts
from identical float32-rounded inputs, relative L2 <= 1e-5 on P, u and S for
float32 storage; walls on all faces (corners, where diagonal links cross two
faces), a periodic axis beside walls, fully periodic with a zero-mean
pressure source, the manufactured problem with time-dependent sources,
16-bit storage with format-derived bounds, the mass ledger and checkpoints."""
import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, gpu_solver, mean_free, oracle_solver, rel_l2, smooth_state
from tests.test_gpu_parity import TOL, _check_fields, _np, reduced_tolerance

pytestmark = pytest.mark.gpu

BETA = 0.2        # inside [max(phi)/2, 2 min(phi)] for phi in [0.15, 0.3] (eq. 3-4)


def q9_params(shape, bc_f=None, bc_g=None):
    p, _ = inputs.injection_problem(shape, 1.0, 4.0, 11, 12)
    p = dict(p, lattice="D2Q9", beta=BETA)
    if bc_f is not None:
        p["bc_f"], p["bc_g"] = bc_f, bc_g
    return p


def q9_pair(params, seed, storage="fp32", Fp=None):
    nx, ny, _ = params["shape"]
    fshape = (1, ny, nx)
    K = f32(5 / 6 * np.exp(inputs.gaussian_random_field((ny, nx), 4.0, seed)).reshape(fshape))
    phi = f32(inputs.uniform_field(fshape, 0.15, 0.3, seed + 1))
    P0, S0 = smooth_state(fshape, seed + 2)
    P0, S0 = f32(P0), f32(S0)
    o = oracle_solver(params, m=64)
    o.set_fields(K, phi, Fp=Fp)
    o.set_state(P0, S0)
    g = gpu_solver(params, m=64, storage=storage)
    g.set_fields(K, phi, Fp=Fp)
    g.set_state(P0, S0)
    return o, g


def replay(o, g, iters, periodic=False, tol=None, what=""):
    s_change = 0.0
    for n, it in enumerate(iters):
        o.update_coefficients()
        g.update_coefficients()
        k_o, _, _ = o.pressure_solve(-1.0, it)
        k_g, _, _ = g.pressure_solve(-1.0, it)
        assert k_o == k_g == it
        t = tol(o, s_change) if tol else None
        _check_fields(o, g, f"D2Q9 {what} step {n}", periodic=periodic, tol=t)
        S_before = o.saturation()
        o.saturation_step()
        g.saturation_step()
        s_change += rel_l2(S_before, o.saturation())


@pytest.mark.parametrize("shape", [(70, 45), (33, 20), (64, 8)])
def test_d2q9_walls_replay(shape):
    params = q9_params(shape)
    o, g = q9_pair(params, seed=sum(shape))
    replay(o, g, [1, 10, 100], what=f"walls {shape}")
    fg, gg = g.populations()
    assert rel_l2(o.f[1:], _np(fg)) <= TOL
    assert rel_l2(o.g, _np(gg)) <= TOL


def test_d2q9_periodic_axis_beside_walls():
    """x periodic, y walls (Dirichlet pressure, Dirichlet / no-flux saturation):
    diagonal links at the y walls wrap in x and reflect in y."""
    bc_f = [("periodic",), ("periodic",), ("abb", 1.0), ("abb", 0.2)]
    bc_g = [("periodic",), ("periodic",), ("abb", 0.9), ("bb",)]
    params = q9_params((40, 24), bc_f, bc_g)
    o, g = q9_pair(params, seed=3)
    replay(o, g, [1, 30, 100], what="periodic x")


def test_d2q9_fully_periodic_with_source():
    params = q9_params((36, 28), [("periodic",)] * 4, [("periodic",)] * 4)
    Fp = inputs.gaussian_random_field((28, 36), 3.0, 77).reshape(1, 28, 36) * 1e-3
    Fp = f32(Fp - Fp.mean())
    Fp = Fp - Fp.mean()
    o, g = q9_pair(params, seed=4, Fp=Fp)
    replay(o, g, [3, 64, 200], periodic=True, what="periodic")


def test_d2q9_manufactured_replay():
    params, mp = inputs.manufactured_problem(48)
    params = dict(params, lattice="D2Q9")
    n = 48 * 48
    o = oracle_solver(params, m=1)
    g = gpu_solver(params)
    src0 = [f32(a) for a in mp.sources(0.0)]
    o.set_fields(mp.K, mp.phi, *src0)
    g.set_fields(np.full(n, mp.K), np.full(n, mp.phi), *src0)
    P0, S0 = f32(mp.P()), f32(mp.S(0.0))
    dP, dS = f32(mp.gradP()), f32(mp.gradS(0.0))
    o.set_state(P0, S0, dP0=dP, dS0=dS)
    g.set_state(P0, S0, dP0=dP[:2], dS0=dS[:2])
    for step in range(8):
        srcs = [f32(a) for a in mp.sources(float(step))]
        o.set_sources(*srcs)
        g.set_sources(*srcs)
        o.update_coefficients()
        g.update_coefficients()
        k, _, _ = o.pressure_solve(1e-10, 100000)
        kg, _, _ = g.pressure_solve(-1.0, k)
        assert kg == k
        if step in (0, 7):
            _check_fields(o, g, f"D2Q9 manufactured step {step}", periodic=True)
        o.saturation_step()
        g.saturation_step()


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_d2q9_reduced_precision_replay(storage):
    params = q9_params((48, 30))
    o, g = q9_pair(params, seed=8, storage=storage)
    replay(o, g, [1, 10, 100, 400], tol=lambda o_, s: reduced_tolerance(o_, storage, s), what=storage)


def test_d2q9_mass_ledger_and_checkpoint():
    params = q9_params((40, 30))
    o, g = q9_pair(params, seed=12)
    g.update_coefficients()
    m0, l0 = g.mass()
    its, _ = g.step(4, -1.0, 40)
    assert its == [40] * 4
    for _ in range(4):
        o.step(-1.0, 40)
    m1, l1 = g.mass()
    mo, lo = o.mass()
    assert abs((m1 - m0) - l1) <= 1e-5 * abs(m0)
    assert abs(m1 - mo) <= TOL * abs(mo)
    assert abs(l1 - lo) <= 1e-4 * max(abs(lo), 1e-3 * abs(mo))
    # checkpoint, run on, restore, run again: bitwise equal
    state = g.get_state()
    g.step(2, -1.0, 40)
    P1 = g.pressure().clone()
    g.put_state(state)
    g.step(2, -1.0, 40)
    assert bool((g.pressure() == P1).all())
