"""The multiple-relaxation-time collision of the D2Q9 pressure lattice on the
GPU against the float64 oracle (which applies the full 9 x 9 M^-1 S M with
the rest population, where the GPU uses the reduced flux/stress form without
it), through the C ABI: replays of the oracle's iteration counts, relative
L2 <= 1e-5 on P, u and S for float32 storage, on both D2Q9 sweep kernels,
walls on every face, a periodic box with a zero-mean source, and 16-bit
storage within its format bound; all rates equal reproduces BGK."""
import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, gpu_solver, mean_free, rel_l2
from tests.test_gpu_d2q9 import q9_pair, q9_params, replay
from tests.test_gpu_parity import reduced_tolerance

pytestmark = pytest.mark.gpu

MRT = ("mrt", 1.4, 1.7, 0.6)


@pytest.mark.parametrize("shape", [(70, 45), (64, 40)])
def test_mrt_walls_replay(shape):
    params = dict(q9_params(shape), collision=MRT)
    o, g = q9_pair(params, seed=sum(shape) + 1)
    replay(o, g, [1, 10, 100], what=f"MRT walls {shape}")


def test_mrt_periodic_with_source_replay():
    bc = [("periodic",)] * 4
    params = dict(q9_params((48, 32), bc, bc), collision=MRT)
    fshape = (1, 32, 48)
    Fp = f32(mean_free(inputs.gaussian_random_field((32, 48), 5.0, 9)).reshape(fshape) * 1e-3)
    o, g = q9_pair(params, seed=21, Fp=Fp)
    replay(o, g, [1, 40, 200], periodic=True, what="MRT periodic")


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_mrt_16bit_within_format_bound(storage):
    params = dict(q9_params((64, 40)), collision=MRT)
    o, g = q9_pair(params, seed=33, storage=storage)
    replay(o, g, [1, 10, 100], tol=lambda o_, s_change: reduced_tolerance(o_, storage, s_change),
           what=f"MRT {storage}")


def test_mrt_equal_rates_is_bgk_on_the_gpu():
    """Uniform K and S give one 1/tau_f; MRT with every rate equal to it must
    match the BGK run (the two forms round differently, so to 1e-6)."""
    params = q9_params((64, 40))
    nx, ny = 64, 40
    fshape = (1, ny, nx)
    K = np.ones(fshape)
    phi = f32(np.full(fshape, 0.25))
    x = (np.arange(nx) + 0.5) / nx
    P0 = f32(np.broadcast_to(1.0 - x, fshape))
    S0 = f32(np.full(fshape, 0.3))
    gb = gpu_solver(params)
    gb.set_fields(K, phi)
    gb.set_state(P0, S0)
    gb.update_coefficients()
    # 1/tau_f at S = 0.3, K = 1 (eq. 2-9, 2-16, 3-11a; c = dt = 1, c_s^2 = 1/3)
    Dp = 0.3 ** 2 / params["mu_w"] + 0.7 ** 2 / params["mu_n"]
    s = 1.0 / (0.5 + 3.0 * Dp)
    gm = gpu_solver(dict(params, collision=("mrt", s, s, s)))
    gm.set_fields(K, phi)
    gm.set_state(P0, S0)
    gm.update_coefficients()
    gb.pressure_solve(-1.0, 300)
    gm.pressure_solve(-1.0, 300)
    err = rel_l2(gb.pressure().cpu().numpy(), gm.pressure().cpu().numpy())
    print("MRT with equal rates vs BGK on the GPU:", err)
    assert err <= 1e-6
    assert rel_l2(gb.velocity().cpu().numpy(), gm.velocity().cpu().numpy()) <= 1e-5


def test_mrt_five_spot_replay():
    """MRT with per-link wall conditions (the five-spot wells), blocked sweeps."""
    from tests.lbhelp import oracle_solver
    from tests.test_gpu_parity import _check_fields
    params, fl = inputs.five_spot(32)
    params = dict(params, collision=MRT)
    o = oracle_solver(params, m=64)
    g = gpu_solver(params, m=64)
    for s in (o, g):
        s.set_fields(f32(fl["K"]), f32(fl["phi"]))
        s.set_state(f32(fl["P0"]), f32(fl["S0"]))
    for n, k in enumerate([1024, 128, 128]):
        o.update_coefficients()
        g.update_coefficients()
        o.pressure_solve(-1.0, k)
        assert g.pressure_solve(-1.0, k)[0] == k
        _check_fields(o, g, f"MRT five-spot step {n}")
        o.saturation_step()
        g.saturation_step()
