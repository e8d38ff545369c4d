"""Parity at the benchmark sizes, in the benchmark's launch configuration
(4096^2 D2Q5 and 512^3 D3Q7 heterogeneous injection, m = 64), on sampled
nodes the oracle computes one by one.

After the initialisation (one node of reach: the central differences of the
initial gradients), k pressure iterations (one node each), a saturation step
(one) and a moment (one), a node's value depends only on the nodes within
that many links.  The oracle therefore runs the same sequence on a crop
around each sampled node, wide enough that whatever its artificial crop
faces do cannot reach the centre; crop faces on the real walls keep the real
conditions.  Samples sit at corners, along walls and in the interior."""
import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, gpu_solver, oracle_solver
from tests.test_gpu_parity import UNIT_ROUNDOFF

pytestmark = pytest.mark.gpu

# pressure iterations before and after the saturation step.  From the
# initial state 65 runs the local sweep 0 alone and then a chunk of blocked
# launches (sweeps 1 .. 63, 9 per launch on D2Q5 and D2Q9) and sweep 64
# alone.  After the saturation step the state is in pull form, and on D2Q5
# the second solve of 65 (K2_2D) is a warm benchmark step's: the re-basing
# sweep 0 inside the first of six blocked launches (11, 11, 11, 11, 11, 9
# sweeps), then sweep 64 alone.  D3Q7 runs 20 and 6.
K1_2D, K1_3D, K2, K2_2D = 65, 20, 6, 65


def reach(k1, k2=K2):
    return 1 + k1 + 1 + 1 + k2 + 1 + 2


def _run(solver, k1, k2):
    solver.update_coefficients()
    solver.pressure_solve(-1.0, k1)
    solver.saturation_step()
    solver.update_coefficients()
    solver.pressure_solve(-1.0, k2)


def _crop_params(params, lo, hi, full):
    """Parameters of the crop [lo, hi) (per axis, x first): the real face
    condition where the crop reaches the domain face, bounce-back elsewhere."""
    p = dict(params)
    shape = tuple(h - l for l, h in zip(lo, hi))
    p["shape"] = shape + (1,) * (3 - len(shape))
    bf, bg = list(params["bc_f"]), list(params["bc_g"])
    for a in range(len(lo)):
        if lo[a] > 0:
            bf[2 * a], bg[2 * a] = ("bb",), ("bb",)
        if hi[a] < full[a]:
            bf[2 * a + 1], bg[2 * a + 1] = ("bb",), ("bb",)
    p["bc_f"], p["bc_g"] = bf, bg
    return p


def _check_samples(params, fl, samples, storage, k1, k2=K2):
    full = params["shape"][:3] if params["lattice"] == "D3Q7" else params["shape"][:2]
    R = reach(k1, k2)
    dim = len(full)
    K, phi, P0, S0 = (inputs.f32(fl[k]) for k in ("K", "phi", "P0", "S0"))
    g = gpu_solver(params, m=64, storage=storage)
    g.set_fields(K.ravel(), phi.ravel())
    g.set_state(P0.ravel(), S0.ravel())
    _run(g, k1, k2)
    P = g.pressure().cpu().numpy()
    u = g.velocity().cpu().numpy()
    S = g.saturation().cpu().numpy()
    del g
    worst = {"P": 0.0, "u": 0.0, "S": 0.0}
    uscale = float(np.abs(u).max())
    for pt in samples:                                   # pt = (x, y[, z])
        lo = [max(0, pt[a] - R) for a in range(dim)]
        hi = [min(full[a], pt[a] + R + 1) for a in range(dim)]
        sl = tuple(slice(lo[a], hi[a]) for a in reversed(range(dim)))   # [z][y][x]
        if dim == 2:
            sl = (slice(0, 1),) + sl
        cp = _crop_params(params, lo, hi, full)
        o = oracle_solver(cp, m=64)
        o.set_fields(f32(K[sl]), f32(phi[sl]))
        o.set_state(f32(P0[sl]), f32(S0[sl]))
        _run(o, k1, k2)
        loc = tuple(pt[a] - lo[a] for a in reversed(range(dim)))
        if dim == 2:
            loc = (0,) + loc
        idx = (0,) + tuple(pt[a] for a in reversed(range(dim))) if dim == 2 else tuple(pt[a] for a in (2, 1, 0))
        Po, uo, So = o.pressure()[loc], o.velocity()[(slice(0, dim),) + loc], o.saturation()[loc]
        Pg, ug, Sg = P[idx], u[(slice(None),) + idx], S[idx]
        # errors against the field scales: P and S lie in [0, 1], u against its largest value
        worst["P"] = max(worst["P"], abs(Pg - Po))
        worst["u"] = max(worst["u"], float(np.max(np.abs(ug - uo))) / uscale)
        worst["S"] = max(worst["S"], abs(Sg - So))
    print(params["lattice"], full, storage, {k: f"{v:.2e}" for k, v in worst.items()})
    return worst


def _samples(full, rng, n_interior, R):
    dim = len(full)
    pts = []
    for corner in range(2 ** dim):                       # every corner
        pts.append(tuple(0 if (corner >> a) & 1 == 0 else full[a] - 1 for a in range(dim)))
    for a in range(dim):                                 # a node on each face
        for side in (0, full[a] - 1):
            p = [int(rng.integers(R, full[b] - R)) for b in range(dim)]
            p[a] = side
            pts.append(tuple(p))
    for _ in range(n_interior):
        pts.append(tuple(int(rng.integers(0, full[a])) for a in range(dim)))
    return pts


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_injection_2d_4096_sampled_parity(storage):
    params, fl = inputs.injection_2d(4096)
    rng = np.random.default_rng(17)
    worst = _check_samples(params, fl, _samples((4096, 4096), rng, 4, reach(K1_2D, K2_2D)), storage, K1_2D, K2_2D)
    tol = 1e-5 if storage == "fp32" else 16 * UNIT_ROUNDOFF[storage]
    for k, v in worst.items():
        assert v <= tol, (k, v, tol)


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_injection_3d_512_sampled_parity(storage):
    """512^3 D3Q7 in every storage format: float32 within 1e-5, the 16-bit
    deviation forms within 16 unit roundoffs of their format (the bound of
    the 2-D case: they round once per sweep here)."""
    params, fl = inputs.injection_3d(512)
    rng = np.random.default_rng(19)
    worst = _check_samples(params, fl, _samples((512, 512, 512), rng, 2, reach(K1_3D)), storage, K1_3D)
    tol = 1e-5 if storage == "fp32" else 16 * UNIT_ROUNDOFF[storage]
    for k, v in worst.items():
        assert v <= tol, (k, v, tol)


def test_ensemble_256_sampled_parity():
    """The 256-member ensemble of the ensemble benchmark (sides 128..1024), one
    autotuned, graph-captured coupled step of 64 iterations (ensemble solves
    run whole chunks of m = 64): sampled nodes of members of every size
    against the oracle on crops."""
    import torch
    from paper_1808_07554_amd import lbtp
    members = inputs.ensemble(256)
    dev = torch.device("cuda", 0)
    b = lbtp.Batch([p for p, _ in members], m=64)
    for i, (p, fl) in enumerate(members):
        d = {k: torch.from_numpy(inputs.f32(fl[k]).ravel()).to(dev) for k in ("K", "phi", "P0", "S0")}
        b.set_fields(i, d["K"], d["phi"])
        b.set_state(i, d["P0"], d["S0"])
    b.autotune(sweeps=3)
    kb = 64
    its, _ = b.step(1, -1.0, kb)
    assert (its[0] == kb).all()
    reach = 1 + kb + 2 + 1 + 2
    rng = np.random.default_rng(23)
    by_size = {}
    for i, (p, _) in enumerate(members):
        by_size.setdefault(p["shape"][0], []).append(i)
    worst = {"P": 0.0, "u": 0.0, "S": 0.0}
    for n, idx in sorted(by_size.items()):
        for i in (idx[0], idx[-1]):
            params, fl = members[i]
            P = b.pressure(i).cpu().numpy()
            u = b.velocity(i).cpu().numpy()
            S = b.saturation(i).cpu().numpy()
            uscale = float(np.abs(u).max())
            for pt in [(0, 0), (n - 1, n - 1), (int(rng.integers(0, n)), int(rng.integers(0, n)))]:
                lo = [max(0, pt[a] - reach) for a in range(2)]
                hi = [min(n, pt[a] + reach + 1) for a in range(2)]
                sl = (slice(0, 1), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
                o = oracle_solver(_crop_params(params, lo, hi, (n, n)), m=64)
                K, phi, P0, S0 = (inputs.f32(fl[k]) for k in ("K", "phi", "P0", "S0"))
                o.set_fields(f32(K[sl]), f32(phi[sl]))
                o.set_state(f32(P0[sl]), f32(S0[sl]))
                o.step(-1.0, kb)
                loc = (0, pt[1] - lo[1], pt[0] - lo[0])
                gidx = (0, pt[1], pt[0])
                worst["P"] = max(worst["P"], abs(P[gidx] - o.pressure()[loc]))
                worst["u"] = max(worst["u"], float(np.max(np.abs(u[(slice(None),) + gidx] -
                                                                 o.velocity()[(slice(0, 2),) + loc]))) / uscale)
                worst["S"] = max(worst["S"], abs(S[gidx] - o.saturation()[loc]))
    b.close()
    print("ensemble 256", sorted(by_size), {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= 1e-5, (k, v)
