"""The five-spot problem (Section 4.3, D2Q9, wells as per-link Dirichlet
segments of no-flux walls set through lbtp_set_wall_types) on the GPU.

  * replays of the oracle: 2048 pressure iterations from the initial ramp,
    then coupled steps of 256 iterations each (the slowest pressure mode of
    this layout, a level shift held only by the short well segments, decays
    by about 0.9995 per iteration, so a solve to r <= 1e-8 takes thousands of
    iterations per step) from the same float32-rounded inputs; P, u and S
    within relative L2 1e-5 for float32 storage (16-bit storage within its
    format-derived bound), on the 4-nodes per thread sweep (N = 32) and the
    one-node sweep (N = 30);
  * a longer run on the GPU alone (N = 64 to T = 1): the saturation stays in
    [0, 1], the solution keeps the layout's x <-> y symmetry, and the change
    of water mass equals the flux the walls let in (the ledger).
"""
import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, gpu_solver, oracle_solver, rel_l2
from tests.test_gpu_parity import _check_fields, reduced_tolerance

pytestmark = pytest.mark.gpu


def _pair(N, storage):
    p, fl = inputs.five_spot(N)
    o = oracle_solver(p, m=64)
    g = gpu_solver(p, m=64, storage=storage)
    for s in (o, g):
        s.set_fields(f32(fl["K"]), f32(fl["phi"]))
        s.set_state(f32(fl["P0"]), f32(fl["S0"]))
    return o, g


@pytest.mark.parametrize("N,storage", [(32, "fp32"), (30, "fp32"), (32, "fp16")])
def test_five_spot_replays_oracle(N, storage):
    o, g = _pair(N, storage)
    s_change, total = 0.0, 0
    for n in range(10):
        o.update_coefficients()
        g.update_coefficients()
        k, _, _ = o.pressure_solve(-1.0, 2048 if n == 0 else 256)
        kg, _, _ = g.pressure_solve(-1.0, k)
        assert kg == k
        total += k
        tol = None if storage == "fp32" else reduced_tolerance(o, storage, s_change)
        _check_fields(o, g, f"five-spot N={N} {storage} step {n}", tol=tol)
        S_before = o.saturation()
        o.saturation_step()
        g.saturation_step()
        s_change += rel_l2(S_before, o.saturation())
    m_o, l_o = o.mass()
    m_g, l_g = g.mass()
    print(f"five-spot N={N} {storage}: {total} iterations; mass {m_o:.6f} / {m_g:.6f}, "
          f"ledger {l_o:.6f} / {l_g:.6f}")
    assert abs(l_g - l_o) <= 1e-4 * abs(l_o)
    assert o.saturation().max() > 0.05         # the injector has let water in


def test_five_spot_run_properties():
    from paper_1808_07554_amd import five_spot
    s, params = five_spot.make_solver(64)
    m0, _ = s.mass()
    nsteps = int(round(1.0 / params["dt"]))
    its = [five_spot.coupled_step(s, 1e-8, 20000) for _ in range(nsteps)]
    s.update_coefficients()
    S = s.saturation().cpu().numpy()[0].astype(np.float64)
    P = s.pressure().cpu().numpy()[0].astype(np.float64)
    m1, ledger = s.mass()
    print(f"five-spot N=64 to T=1: {nsteps} steps, {sum(its)} iterations (first {its[0]}), "
          f"S in [{S.min():.3e}, {S.max():.4f}], mass {m0:.4f} -> {m1:.4f}, ledger {ledger:.4f}")
    assert -1e-6 <= S.min() and S.max() <= 1.0 + 1e-6
    assert S.max() > 0.5 and S[-1, -1] < S[0, 0]
    assert np.abs(S - S.T).max() <= 1e-4
    assert np.abs(P - P.T).max() <= 1e-5
    d = np.diag(P)
    assert d[0] > d[-1]
    assert abs((m1 - m0) - ledger) <= 1e-4 * abs(ledger)
