"""Ensembles on the GPU: every member of a batched run equals a separate
single-realisation run (bit for bit), and the per-member solves stop on their
own.  (Single-realisation runs are checked against the oracle in
test_gpu_parity.py.)  With float32 storage the blocked plain sweeps equal
single sweeps bit for bit, so both sides run their defaults; with 16-bit
storage a blocked launch rounds to the storage format once, and a single
context runs its last partial chunk one sweep per launch where an ensemble
runs whole chunks, so both sides run one sweep per launch there."""
import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, gpu_solver, oracle_solver, rel_l2

pytestmark = pytest.mark.gpu


def _members(shapes, seed0=70):
    ms = []
    for j, shape in enumerate(shapes):
        p, fl = inputs.injection_problem(shape, 0.5 + 0.3 * j, 4.0, seed0 + 2 * j, seed0 + 2 * j + 1)
        fshape = fl["K"].shape
        S0 = 0.3 + 0.2 * np.tanh(inputs.gaussian_random_field(fshape[1:] if fshape[0] == 1 else fshape, 5.0,
                                                               seed0 + 100 + j)).reshape(fshape)
        fl["S0"] = S0
        ms.append((p, {k: f32(v) for k, v in fl.items()}))
    return ms


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_batch_members_equal_single_runs(storage):
    from paper_1808_07554_amd import lbtp
    shapes = [(32, 32), (64, 40), (128, 24), (36, 60), (100, 8)]
    ms = _members(shapes)
    if storage != "fp32":
        ms = [(dict(p, sweep_block=1), fl) for p, fl in ms]
    b = lbtp.Batch([p for p, _ in ms], m=16, storage=storage)
    singles = []
    for i, (p, fl) in enumerate(ms):
        b.set_fields(i, fl["K"], fl["phi"])
        b.set_state(i, fl["P0"], fl["S0"])
        s = gpu_solver(p, m=16, storage=storage)
        s.set_fields(fl["K"], fl["phi"])
        s.set_state(fl["P0"], fl["S0"])
        singles.append(s)
    # replay: a fixed number of iterations per step
    its, st = b.step(3, -1.0, 48)
    assert (its == 48).all()
    for s in singles:
        s.step(3, -1.0, 48)
    for i, s in enumerate(singles):
        assert bool((b.pressure(i) == s.pressure()).all()), i
        assert bool((b.saturation(i) == s.saturation()).all()), i
        assert bool((b.velocity(i) == s.velocity()).all()), i
        mb, lb = b.mass(i)
        ms_, ls = s.mass()
        assert mb == ms_
        assert abs(lb - ls) <= 1e-12 * max(1.0, abs(ms_))
    # converging steps: each member stops on its own, like its single run
    its_b, _ = b.step(2, 1e-6, 16 * 4000)
    for i, s in enumerate(singles):
        its_s, _ = s.step(2, 1e-6, 16 * 4000)
        assert list(its_b[:, i]) == its_s, (i, its_b[:, i], its_s)
        assert bool((b.pressure(i) == s.pressure()).all()), i
        assert bool((b.saturation(i) == s.saturation()).all()), i
    assert len(set(its_b[0])) > 1          # the members really needed different counts


def test_batch_autotune_keeps_results():
    from paper_1808_07554_amd import lbtp
    shapes = [(64, 64), (128, 32), (32, 96)]
    ms = _members(shapes, seed0=90)

    def run(nt):
        b = lbtp.Batch([p for p, _ in ms], m=16)
        for i, (p, fl) in enumerate(ms):
            b.set_fields(i, fl["K"], fl["phi"])
            b.set_state(i, fl["P0"], fl["S0"])
        if nt == "auto":
            chosen = b.autotune(sweeps=4)
            assert chosen in (64, 128, 256, 512)
        else:
            b.set_threads(nt)
        b.step(2, 1e-7, 16 * 2000)
        return [_np(b.pressure(i)) for i in range(len(ms))] + [_np(b.saturation(i)) for i in range(len(ms))]

    ref = run(256)
    for nt in (64, 512, "auto"):
        got = run(nt)
        for a, c in zip(ref, got):
            assert np.array_equal(a, c), nt


def test_batch_member_against_oracle():
    from paper_1808_07554_amd import lbtp
    ms = _members([(48, 20), (40, 44)], seed0=110)
    b = lbtp.Batch([p for p, _ in ms], m=16)
    for i, (p, fl) in enumerate(ms):
        b.set_fields(i, fl["K"], fl["phi"])
        b.set_state(i, fl["P0"], fl["S0"])
    b.step(3, -1.0, 64)
    for i, (p, fl) in enumerate(ms):
        o = oracle_solver(p, m=16)
        o.set_fields(fl["K"].astype(np.float64), fl["phi"].astype(np.float64))
        o.set_state(fl["P0"].astype(np.float64), fl["S0"].astype(np.float64))
        for _ in range(3):
            o.step(-1.0, 64)
        assert rel_l2(o.pressure(), _np(b.pressure(i))) <= 1e-5
        assert rel_l2(o.saturation(), _np(b.saturation(i))) <= 1e-5
        assert rel_l2(o.velocity()[:2], _np(b.velocity(i))) <= 1e-5


def test_batch_rejects_bad_arguments():
    from paper_1808_07554_amd import lbtp
    ms = _members([(32, 32), (30, 32)])
    with pytest.raises(lbtp.LbtpError):          # nx % 4 != 0
        lbtp.Batch([p for p, _ in ms], m=16)
    ms = _members([(32, 32)])
    with pytest.raises(lbtp.LbtpError):          # odd residual stride
        lbtp.Batch([p for p, _ in ms], m=15)
    b = lbtp.Batch([p for p, _ in ms], m=16)
    with pytest.raises(lbtp.LbtpError) as e:     # step before set_state
        b.step(1, -1.0, 16)
    assert e.value.code == lbtp.ESTATE
    b.set_fields(0, ms[0][1]["K"], ms[0][1]["phi"])
    b.set_state(0, ms[0][1]["P0"], ms[0][1]["S0"])
    with pytest.raises(lbtp.LbtpError):          # max_iters not a multiple of m
        b.step(1, -1.0, 20)


def test_autotuned_tilings_per_size_class_keep_single_run_results():
    """m = 64 and members of three sizes: the autotuner picks, per size class,
    a region shape and an odd block length dividing the 63 plain sweeps of a
    chunk; every member still equals its single-context run bit for bit
    (float32 blocked sweeps equal single sweeps for any shape and block
    length), through solves to a tolerance that take many chunks (the
    ensemble runs them in graphs of several chunks)."""
    from paper_1808_07554_amd import lbtp
    shapes = [(128, 128), (256, 96), (64, 64), (128, 128)]
    ms = _members(shapes, seed0=130)
    b = lbtp.Batch([p for p, _ in ms], m=64)
    singles = []
    for i, (p, fl) in enumerate(ms):
        b.set_fields(i, fl["K"], fl["phi"])
        b.set_state(i, fl["P0"], fl["S0"])
        s = gpu_solver(p, m=64)
        s.set_fields(fl["K"], fl["phi"])
        s.set_state(fl["P0"], fl["S0"])
        singles.append(s)
    b.autotune(sweeps=2)
    shapes_ok = {(8, 8), (8, 6), (16, 4), (4, 8)}
    tilings = [b.tiling(i) for i in range(len(ms))]
    print("tuned tilings (waves, rows per wave, sweeps per launch):", tilings)
    for (w, r, h) in tilings:
        assert (w, r) in shapes_ok and h >= 3 and h % 2 == 1 and 63 % h == 0
        assert w * r - 2 * h >= 16 and 64 - 2 * h >= 16
    assert tilings[0] == tilings[3]              # one class per size
    its_b, _ = b.step(3, 1e-7, 64 * 400)
    assert its_b[0].max() > 4 * 64               # the first solve took several chunks
    for i, s in enumerate(singles):
        its_s, _ = s.step(3, 1e-7, 64 * 400)
        assert list(its_b[:, i]) == its_s, (i, its_b[:, i], its_s)
        assert bool((b.pressure(i) == s.pressure()).all()), i
        assert bool((b.saturation(i) == s.saturation()).all()), i
        assert bool((b.velocity(i) == s.velocity()).all()), i


@pytest.mark.parametrize("kind,storage", [("D2Q9", "fp32"), ("D2Q9", "fp16"), ("capillary", "fp32"),
                                          ("D2Q9-capillary", "bf16")])
def test_d2q9_and_capillary_members_equal_single_runs(kind, storage):
    """Ensembles of the paper's D2Q9 lattice (beta inside the eq. 3-4 bounds)
    and of members with the capillary diffusivity field D_s(S, x) (a tau_g
    per node): every member equals its single-context run bit for bit, with
    fixed iteration counts and with solves to a tolerance (one sweep per
    launch on both sides for 16-bit storage, as in the other ensemble test)."""
    from paper_1808_07554_amd import lbtp
    shapes = [(32, 32), (64, 40), (48, 24)]
    ms = _members(shapes, seed0=150)
    ms = [(dict(p, lattice="D2Q9" if kind.startswith("D2Q9") else p["lattice"],
                beta=0.2 if kind.startswith("D2Q9") else p["beta"],
                cap_B=0.05 if kind.endswith("capillary") else 0.0,
                **({} if storage == "fp32" else {"sweep_block": 1})), fl) for p, fl in ms]
    b = lbtp.Batch([p for p, _ in ms], m=16, storage=storage)
    singles = []
    for i, (p, fl) in enumerate(ms):
        b.set_fields(i, fl["K"], fl["phi"])
        b.set_state(i, fl["P0"], fl["S0"])
        s = gpu_solver(p, m=16, storage=storage)
        s.set_fields(fl["K"], fl["phi"])
        s.set_state(fl["P0"], fl["S0"])
        singles.append(s)
    its, _ = b.step(2, -1.0, 48)
    assert (its == 48).all()
    its_b, _ = b.step(2, 1e-6, 16 * 2000)
    for i, s in enumerate(singles):
        s.step(2, -1.0, 48)
        its_s, _ = s.step(2, 1e-6, 16 * 2000)
        assert list(its_b[:, i]) == its_s, (i, its_b[:, i], its_s)
        assert bool((b.pressure(i) == s.pressure()).all()), i
        assert bool((b.saturation(i) == s.saturation()).all()), i
        assert bool((b.velocity(i) == s.velocity()).all()), i
