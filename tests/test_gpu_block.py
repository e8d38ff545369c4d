"""Temporal blocking of the plain pressure sweeps (several sweeps per launch,
the region held in registers on D2Q5 and D2Q9, streaming along z on D3Q7)
against one sweep per launch, through the C ABI.

With float32 storage the blocked launches perform the same arithmetic in the
same order, so populations, pressure and saturation must agree bitwise: on
walled, periodic and mixed boxes, boxes narrower than a tile or than the
halo, ragged tile counts, per-link Dirichlet data, a pressure source and
every block length.  16-bit storage rounds to its format once per launch
instead of once per sweep, so there the blocked path must stay within the
format's bound of the one-sweep path.  D2Q9 adds corners (the y face's rule),
diagonals that wrap across a periodic axis beside a wall, per-link wall data
and conditions (the five-spot) and the MRT collision.  The oracle parity of
the blocked path itself is covered by every other D2Q5 and D2Q9 test, which
run it by default."""
import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, gpu_solver, mean_free, smooth_state
from tests.test_gpu_parity import UNIT_ROUNDOFF

pytestmark = pytest.mark.gpu

WALLS = ([("abb", 1.0), ("abb", 0.0), ("bb",), ("bb",)], [("abb", 1.0), ("outflow",), ("bb",), ("bb",)])
PERIODIC = ([("periodic",)] * 4, [("periodic",)] * 4)
MIXED = ([("periodic",), ("periodic",), ("abb", 0.7), ("abb", 0.2)],
         [("periodic",), ("periodic",), ("abb", 0.9), ("bb",)])


def _run(shape, bcs, sweep_block, storage="fp32", Fp=False, wall_face=None, iters=(200, 130)):
    nx, ny = shape
    params, _ = inputs.injection_problem(shape, 1.0, 4.0, 11, 12)
    params = dict(params, bc_f=bcs[0], bc_g=bcs[1])
    fshape = (1, ny, nx)
    K = f32(np.exp(inputs.gaussian_random_field((ny, nx), 4.0, nx + ny)).reshape(fshape) * params["mu_n"] / 6)
    phi = f32(inputs.uniform_field(fshape, 0.15, 0.3, 7))
    P0, S0 = (f32(a) for a in smooth_state(fshape, 5))
    fp = f32(mean_free(np.sin(np.arange(nx * ny) * 0.37)) * 1e-3).reshape(fshape) if Fp else None
    g = gpu_solver(params, m=64, storage=storage, sweep_block=sweep_block)
    g.set_fields(K, phi, Fp=fp)
    g.set_state(P0, S0)
    if wall_face is not None:
        n_along = ny if wall_face < 2 else nx
        g.set_wall_values(wall_face, P=f32(1.0 + 0.1 * np.cos(np.arange(n_along) * 0.2)))
    for n, k in enumerate(iters):
        g.update_coefficients()
        assert g.pressure_solve(-1.0, k)[0] == k
        if n + 1 < len(iters):
            g.saturation_step()
    f, gg = g.populations()
    out = dict(f=f.cpu().numpy(), g=gg.cpu().numpy(), P=g.pressure().cpu().numpy(), S=g.saturation().cpu().numpy())
    g.close()
    return out


CASES = [
    ((200, 150), WALLS, {}),
    ((64, 64), PERIODIC, dict(Fp=True)),
    ((20, 12), PERIODIC, dict(Fp=True)),         # narrower than the halo: the region wraps several times
    ((130, 70), MIXED, {}),
    ((96, 47), WALLS, dict(wall_face=0)),
    ((90, 40), MIXED, dict(wall_face=2)),         # per-link data along a periodic axis
    ((300, 7), WALLS, {}),
    ((7, 300), MIXED, {}),
    ((150, 90), WALLS, dict(Fp=True)),            # a pressure source with walls on every face
    ((90, 60), MIXED, dict(Fp=True, wall_face=2)),
    # the smallest boxes: walled axes of 3 nodes, periodic axes of 1 and 2
    ((3, 3), WALLS, dict(wall_face=1)),
    ((3, 41), WALLS, dict(wall_face=0)),
    ((1, 33), MIXED, {}),
    ((2, 2), PERIODIC, dict(Fp=True)),
    # grids of many tiles, where launches without a source take regions of 9 rows per wavefront
    ((1024, 1024), WALLS, {}),
    ((1100, 1050), MIXED, dict(wall_face=2)),
]


@pytest.mark.parametrize("shape,bcs,kw", CASES)
def test_blocked_sweeps_bitwise_equal_single_sweeps(shape, bcs, kw):
    ref = _run(shape, bcs, 1, **kw)
    got = _run(shape, bcs, 9, **kw)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), (shape, k, float(np.abs(ref[k] - got[k]).max()))


def test_fixed_count_solves_ending_on_a_chunk_bitwise():
    """Solves of a whole number of chunks without the stopping rule: the
    last chunk runs as blocked launches too (it ends at sweep jm - 1)."""
    ref = _run((200, 150), WALLS, 1, iters=(640, 128))
    got = _run((200, 150), WALLS, 9, iters=(640, 128))
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k


@pytest.mark.parametrize("H", [3, 5, 7, 21, 23])
def test_every_block_length_bitwise(H):
    ref = _run((150, 110), WALLS, 1)
    got = _run((150, 110), WALLS, H)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), (H, k)


def _run_checked(shape, bcs, sweep_block, m=64, Fp=False, tol=1e-7, steps=3):
    """Solves with the stopping rule on: the first from the initial state
    (local form: sweep 0 in a launch of its own), the later ones warm (pull
    form: every chunk's re-basing sweep inside its first blocked launch)."""
    nx, ny = shape
    params, _ = inputs.injection_problem(shape, 1.0, 4.0, 11, 12)
    params = dict(params, bc_f=bcs[0], bc_g=bcs[1])
    fshape = (1, ny, nx)
    K = f32(np.exp(inputs.gaussian_random_field((ny, nx), 4.0, nx + ny)).reshape(fshape) * params["mu_n"] / 6)
    phi = f32(inputs.uniform_field(fshape, 0.15, 0.3, 7))
    P0, S0 = (f32(a) for a in smooth_state(fshape, 5))
    fp = f32(mean_free(np.sin(np.arange(nx * ny) * 0.37)) * 1e-3).reshape(fshape) if Fp else None
    g = gpu_solver(params, m=m, sweep_block=sweep_block)
    g.set_fields(K, phi, Fp=fp)
    g.set_state(P0, S0)
    solves = []
    for n in range(steps):
        g.update_coefficients()
        solves.append(g.pressure_solve(tol, 10_000_000))
        if n + 1 < steps:
            g.saturation_step()
    f, gg = g.populations()
    out = dict(f=f.cpu().numpy(), g=gg.cpu().numpy(), P=g.pressure().cpu().numpy(), S=g.saturation().cpu().numpy())
    g.close()
    return solves, out


CHECKED = [
    ((200, 150), WALLS, 9, 64, {}),
    ((130, 70), MIXED, 9, 64, dict(Fp=True)),
    ((64, 64), PERIODIC, 9, 64, dict(Fp=True, tol=1e-9)),
    ((150, 110), WALLS, 23, 64, {}),     # chunks of 17 + 17 + 15 + 15 sweeps (21 + 21 + 21 after sweep 0)
    ((150, 110), WALLS, 3, 64, {}),
    ((96, 47), WALLS, 9, 8, {}),         # short chunks: 5 + 3 sweeps (one launch of 7 after sweep 0)
    ((20, 12), PERIODIC, 9, 6, dict(Fp=True)),   # 3 + 3 sweeps, narrower than the halo
    ((1024, 1024), WALLS, 9, 64, dict(steps=2)),  # regions of 9 rows per wavefront
]


@pytest.mark.parametrize("shape,bcs,H,m,kw", CHECKED)
def test_checked_solves_blocked_equal_single_sweeps(shape, bcs, H, m, kw):
    """The re-basing sweep of a chunk runs inside its first blocked launch
    and the stopping rule is evaluated by a probe at the end of its last one:
    same stopping iterations, bitwise the same state, and the residual up to
    the order of its float64 sums."""
    ref_solves, ref = _run_checked(shape, bcs, 1, m=m, **kw)
    got_solves, got = _run_checked(shape, bcs, H, m=m, **kw)
    print(shape, H, m, [(k, f"{r:.3e}") for k, r, _ in got_solves])
    for (k0, r0, st0), (k1, r1, st1) in zip(ref_solves, got_solves):
        assert (k0, st0) == (k1, st1), (ref_solves, got_solves)
        assert abs(r1 - r0) <= 1e-12 * abs(r0), (r0, r1)
    assert len(ref_solves[0]) and ref_solves[0][0] > m     # the cold solve runs several chunks
    for k in ref:
        assert np.array_equal(ref[k], got[k]), (shape, k, float(np.abs(ref[k] - got[k]).max()))


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_blocked_16bit_within_format_bound(storage):
    ref = _run((200, 150), WALLS, 1, storage=storage)
    got = _run((200, 150), WALLS, 9, storage=storage)
    ur = UNIT_ROUNDOFF[storage]
    for k in ("P", "S"):
        err = float(np.abs(ref[k] - got[k]).max())
        print(storage, k, f"{err:.2e}")
        assert err <= 16 * ur, (storage, k, err)


# ----------------------------------------------------------------- D2Q9
def _run_q9(shape, bcs, sweep_block, storage="fp32", Fp=False, wall_face=None, collision=None, params=None,
            fields=None, iters=(200, 130)):
    nx, ny = shape
    if params is None:
        params, _ = inputs.injection_problem(shape, 1.0, 4.0, 11, 12)
        params = dict(params, lattice="D2Q9", beta=0.2, bc_f=bcs[0], bc_g=bcs[1])
    if collision is not None:
        params = dict(params, collision=collision)
    fshape = (1, ny, nx)
    if fields is None:
        K = f32(np.exp(inputs.gaussian_random_field((ny, nx), 4.0, nx + ny)).reshape(fshape) * params["mu_n"] / 6)
        phi = f32(inputs.uniform_field(fshape, 0.15, 0.3, 7))
        P0, S0 = (f32(a) for a in smooth_state(fshape, 5))
    else:
        K, phi, P0, S0 = (f32(fields[k]) for k in ("K", "phi", "P0", "S0"))
    fp = f32(mean_free(np.sin(np.arange(nx * ny) * 0.37)) * 1e-3).reshape(fshape) if Fp else None
    g = gpu_solver(params, m=64, storage=storage, sweep_block=sweep_block)
    g.set_fields(K, phi, Fp=fp)
    g.set_state(P0, S0)
    if wall_face is not None:
        n_along = ny if wall_face < 2 else nx
        g.set_wall_values(wall_face, P=f32(1.0 + 0.1 * np.cos(np.arange(3 * n_along) * 0.2)))
    for n, k in enumerate(iters):
        g.update_coefficients()
        assert g.pressure_solve(-1.0, k)[0] == k
        if n + 1 < len(iters):
            g.saturation_step()
    f, gg = g.populations()
    out = dict(f=f.cpu().numpy(), g=gg.cpu().numpy(), P=g.pressure().cpu().numpy(), S=g.saturation().cpu().numpy())
    g.close()
    return out


Q9_WALLS = ([("abb", 1.0), ("abb", 0.0), ("bb",), ("abb", 0.4)], [("abb", 1.0), ("outflow",), ("bb",), ("bb",)])

Q9_CASES = [
    ((200, 150), Q9_WALLS, {}),                                   # corners: the y face decides
    ((64, 64), PERIODIC, dict(Fp=True)),
    ((20, 12), PERIODIC, dict(Fp=True)),
    ((130, 70), MIXED, {}),                                       # diagonals wrap in x, reflect in y
    ((96, 47), Q9_WALLS, dict(wall_face=0)),                      # per-link wall data, three slots
    ((90, 40), MIXED, dict(wall_face=3)),
    ((7, 300), MIXED, {}),
    ((200, 150), Q9_WALLS, dict(collision=("mrt", 1.4, 1.7, 0.6))),
    ((130, 70), Q9_WALLS, dict(Fp=True)),
    ((130, 70), Q9_WALLS, dict(Fp=True, collision=("mrt", 1.4, 1.7, 0.6))),
    ((3, 3), Q9_WALLS, dict(wall_face=1)),
    ((1, 29), MIXED, {}),
    ((2, 2), PERIODIC, dict(Fp=True)),
    ((1024, 1024), Q9_WALLS, {}),                                 # regions of 5 rows per wavefront
    ((1030, 1000), MIXED, dict(wall_face=3)),
]


@pytest.mark.parametrize("shape,bcs,kw", Q9_CASES)
def test_q9_blocked_sweeps_bitwise_equal_single_sweeps(shape, bcs, kw):
    ref = _run_q9(shape, bcs, 1, **kw)
    got = _run_q9(shape, bcs, 9, **kw)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), (shape, k, float(np.abs(ref[k] - got[k]).max()))


def test_q9_five_spot_blocked_bitwise():
    """Per-link wall conditions (wells in no-flux walls) on the blocked path."""
    params, fl = inputs.five_spot(96)
    ref = _run_q9((96, 96), None, 1, params=params, fields=fl, iters=(300, 128))
    got = _run_q9((96, 96), None, 9, params=params, fields=fl, iters=(300, 128))
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k


@pytest.mark.parametrize("H", [3, 5, 7, 21, 23])
def test_q9_every_block_length_bitwise(H):
    ref = _run_q9((150, 110), Q9_WALLS, 1)
    got = _run_q9((150, 110), Q9_WALLS, H)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), (H, k)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_q9_blocked_16bit_within_format_bound(storage):
    ref = _run_q9((200, 150), Q9_WALLS, 1, storage=storage)
    got = _run_q9((200, 150), Q9_WALLS, 9, storage=storage)
    ur = UNIT_ROUNDOFF[storage]
    for k in ("P", "S"):
        err = float(np.abs(ref[k] - got[k]).max())
        print("D2Q9", storage, k, f"{err:.2e}")
        assert err <= 16 * ur, (storage, k, err)


# ----------------------------------------------------------------- D3Q7
# The z-streaming kernel (H = 3): columns of 64 x 16 nodes walking segments of
# z, walls applied in place on every face.
def _run3(shape, bcs, sweep_block, storage="fp32", Fp=False, wall_face=None, iters=(130, 67)):
    nx, ny, nz = shape
    params, _ = inputs.injection_problem(shape, 1.0, 4.0, 11, 12)
    params = dict(params, bc_f=bcs[0], bc_g=bcs[1])
    fshape = (nz, ny, nx)
    K = f32(np.exp(inputs.gaussian_random_field(fshape, 3.0, nx + ny + nz)) * params["mu_n"] / 8)
    phi = f32(inputs.uniform_field(fshape, 0.15, 0.3, 7))
    P0, S0 = (f32(a) for a in smooth_state(fshape, 5))
    fp = f32(mean_free(np.sin(np.arange(nx * ny * nz) * 0.37)) * 1e-3).reshape(fshape) if Fp else None
    g = gpu_solver(params, m=64, storage=storage, sweep_block=sweep_block)
    g.set_fields(K, phi, Fp=fp)
    g.set_state(P0, S0)
    if wall_face is not None:
        n_face = nx * ny * nz // shape[wall_face // 2]
        g.set_wall_values(wall_face, P=f32(1.0 + 0.1 * np.cos(np.arange(n_face) * 0.2)))
    for n, k in enumerate(iters):
        g.update_coefficients()
        assert g.pressure_solve(-1.0, k)[0] == k
        if n + 1 < len(iters):
            g.saturation_step()
    f, gg = g.populations()
    out = dict(f=f.cpu().numpy(), g=gg.cpu().numpy(), P=g.pressure().cpu().numpy(), S=g.saturation().cpu().numpy())
    g.close()
    return out


WALLS3 = ([("abb", 1.0), ("abb", 0.0)] + [("bb",)] * 4, [("abb", 1.0), ("outflow",)] + [("bb",)] * 4)
PERIODIC3 = ([("periodic",)] * 6, [("periodic",)] * 6)
MIXED3 = ([("periodic",), ("periodic",), ("abb", 0.7), ("abb", 0.2), ("bb",), ("abb", 0.5)],
          [("periodic",), ("periodic",), ("abb", 0.9), ("bb",), ("bb",), ("bb",)])
ZPER3 = ([("abb", 1.0), ("bb",), ("bb",), ("abb", 0.3), ("periodic",), ("periodic",)],
         [("abb", 1.0), ("outflow",), ("bb",), ("bb",), ("periodic",), ("periodic",)])

Q7_CASES = [
    ((40, 30, 20), WALLS3, {}),
    ((70, 23, 18), PERIODIC3, dict(Fp=True)),      # two columns in x, two in y
    ((20, 12, 9), PERIODIC3, dict(Fp=True)),       # narrower than the halo: columns wrap
    ((130, 25, 33), MIXED3, {}),                   # three columns in x, three segments in z
    ((33, 40, 70), ZPER3, {}),                     # a periodic z walked in five segments
    ((45, 28, 19), WALLS3, dict(wall_face=0)),     # per-link data on an x face
    ((45, 28, 19), MIXED3, dict(wall_face=5)),     # ... on a z face
    ((38, 21, 17), ZPER3, dict(wall_face=3)),      # ... on a y face beside a periodic z
    ((50, 30, 24), WALLS3, dict(Fp=True)),
    ((3, 3, 3), WALLS3, dict(wall_face=1)),
    ((1, 5, 33), MIXED3, {}),
    ((2, 2, 2), PERIODIC3, dict(Fp=True)),
]


@pytest.mark.parametrize("shape,bcs,kw", Q7_CASES)
def test_q7_blocked_sweeps_bitwise_equal_single_sweeps(shape, bcs, kw):
    ref = _run3(shape, bcs, 1, **kw)
    got = _run3(shape, bcs, 3, **kw)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), (shape, k, float(np.abs(ref[k] - got[k]).max()))


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_q7_blocked_16bit_within_format_bound(storage):
    ref = _run3((40, 30, 20), WALLS3, 1, storage=storage)
    got = _run3((40, 30, 20), WALLS3, 3, storage=storage)
    ur = UNIT_ROUNDOFF[storage]
    for k in ("P", "S"):
        err = float(np.abs(ref[k] - got[k]).max())
        print("D3Q7", storage, k, f"{err:.2e}")
        assert err <= 16 * ur, (storage, k, err)


def test_q7_block_lengths_other_than_3_rejected():
    from paper_1808_07554_amd import lbtp
    params, _ = inputs.injection_problem((16, 16, 16), 1.0, 4.0, 1, 2)
    for H in (5, 9):
        with pytest.raises(lbtp.LbtpError):
            gpu_solver(params, m=64, sweep_block=H)
