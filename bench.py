"""Benchmark of the coupled two-lattice LB path on one MI355X.

Workload: heterogeneous injection, 2-D 4096 x 4096 on D2Q5, float32
populations, log-normal permeability (seeded Gaussian random field,
sigma_lnK = 1, correlation length 16 cells), porosity uniform in [0.15, 0.3],
quadratic relative permeabilities, viscosity ratio 5, pressure 1 / saturation
1 imposed at x = 0, pressure 0 and a zero-gradient saturation outlet at
x = L, no flux on y faces, S0 = 0, P0 linear.  Every coupled step solves the
pressure lattice to r <= 1e-8 (residual stride m = 64) and advances the
saturation lattice once.

A "step" is one coupled step.  W warm-up steps (the first one is the cold
pressure solve from the linear profile) are followed by K timed steps,
bracketed by torch.cuda.synchronize().  value = MLUPS over both lattices:
cells x (pressure iterations + saturation steps) / time / 1e6.

Also reported: the dominant kernel against its roofline (average launch
duration from HIP events around a burst of launches on the solver's
stream): on D2Q5 and D2Q9 the blocked plain pressure sweep (9 sweeps per
launch through registers, against the vector ALU rate), elsewhere the one-sweep
kernel against HBM; and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1808_07554_amd.profile_sweep import (METHOD_FLOPS_PER_NODE_SWEEP, source_digest,  # noqa: E402
                                                 sweep_kernel_name)

HBM_PEAK_GBS = 8000.0
# vector fp32 rate without packed math (off in this build): one fused
# multiply-add (two flops) per lane per clock, 64 lanes per compute unit, 256
# compute units at 2.4 GHz (the 157.3 TFLOP/s figure counts packed FMA, four
# flops per lane and clock).  The BGK relaxation of the pressure sweeps is one
# FMA per population; the other operations are single adds or multiplies.
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# flops the method itself does in one plain pressure sweep per node (eq. 3-1,
# eq. 3-9a; the count is itemised where it is defined): D2Q5 17, D3Q7 25, D2Q9 34
BLOCK_FLOPS_PER_NODE_SWEEP = METHOD_FLOPS_PER_NODE_SWEEP
# algorithmic bytes of one plain pressure sweep per node: the Q-1 stored
# deviations read and written, 1/tau_f and the base pressure P_b read
POP_BYTES = {"fp32": 4, "fp16": 2, "bf16": 2}


def f_sweep_bytes(lattice, storage):
    q1 = {"D2Q5": 4, "D3Q7": 6, "D2Q9": 8}[lattice]
    return 2 * q1 * POP_BYTES[storage] + 4 + 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "f_block_traffic_injection2d_4096_{}.txt")
TRAFFIC_FILE_Q9 = os.path.join(ROOT, "profiles", "f_block_traffic_injection2d_4096_d2q9_{}.txt")
TRAFFIC_FILE_Q7 = os.path.join(ROOT, "profiles", "f_block_traffic_injection3d_512_{}.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4999)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--m", type=int, default=64)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--workload", default="injection2d", choices=["injection2d", "injection3d", "ensemble", "five-spot"],
                    help="injection2d (default): 4096^2 D2Q5; injection3d: 512^3 D3Q7; ensemble: 256 uneven 2-D "
                         "realisations; five-spot: the Section 4.3 problem on D2Q9 (--n 96 by default)")
    ap.add_argument("--lattice", default="D2Q5", choices=["D2Q5", "D2Q9"],
                    help="lattice of the 2-D injection workload (D2Q9: the paper's own, beta = 0.2)")
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--iters-per-step", type=int, default=64,
                    help="ensemble: pressure iterations per coupled step (fixed, equal work for batched and sequential)")
    ap.add_argument("--max-iters", type=int, default=20_000_000)
    ap.add_argument("--sweep-block", type=int, default=0,
                    help="plain sweeps per blocked launch (0: the library default for the lattice)")
    ap.add_argument("--burst", type=int, default=30, help="launches of the dominant kernel timed for the roofline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tail", action="store_true",
                    help="2-D injection: skip running the rest of the 5000 configured coupled steps")
    ap.add_argument("--no-legs", action="store_true",
                    help="2-D injection: skip the fp16 / bf16 storage legs and the ensemble and warm-start legs")
    return ap.parse_args()


def measured_traffic(storage, lattice="D2Q5"):
    """HBM bytes per f-sweep launch from the committed rocprofv3 counter summary
    for this lattice and storage format, if it was taken on the current kernel
    sources (else None)."""
    path = {"D2Q9": TRAFFIC_FILE_Q9, "D3Q7": TRAFFIC_FILE_Q7}.get(lattice, TRAFFIC_FILE).format(storage)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    b = re.search(r"bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or source_digest(lattice) != m.group(1):
        return None
    return float(b.group(1))


def cpu_baseline(seconds):
    """The float64 oracle on a 512 x 512 crop of the same workload recipe:
    coupled steps with 64 pressure iterations each until ~seconds of CPU work."""
    import oracle
    from paper_1808_07554_amd import inputs
    n = 512
    params, fl = inputs.injection_problem((n, n), 1.0, 16.0, 2, 3)
    o = oracle.Solver(params["lattice"], params["shape"], beta=params["beta"], Ds=params["Ds"],
                      coef=oracle.QuadraticKr(params["mu_w"], params["mu_n"]),
                      bc_f=params["bc_f"], bc_g=params["bc_g"], m=64)
    o.set_fields(inputs.f32(fl["K"]).astype(np.float64), inputs.f32(fl["phi"]).astype(np.float64))
    o.set_state(fl["P0"], fl["S0"])
    t0 = time.perf_counter()
    steps = 0
    while True:
        o.step(-1.0, 64)
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    updates = n * n * steps * (64 + 1)
    return {"value": updates / dt / 1e6, "unit": "MLUPS", "cores": 1, "host_cores": os.cpu_count(), "kind": "oracle",
            "sample": f"float64 NumPy oracle, 512x512 crop of the same recipe, {steps} coupled steps "
                      f"of 64 pressure iterations + 1 saturation step, {dt:.1f} s"}


def ensemble_bench(a):
    """All members advanced together (one launch per kernel per sweep, graph-captured
    chunks) against the same members run one after another through single
    contexts, at a fixed number of pressure iterations per coupled step."""
    import torch
    from paper_1808_07554_amd import inputs, lbtp

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    members = inputs.ensemble(a.members)
    print(f"ensemble inputs: {len(members)} members, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    cells = sum(p["shape"][0] * p["shape"][1] for p, _ in members)
    it = a.iters_per_step
    b = lbtp.Batch([p for p, _ in members], m=a.m, storage=a.storage)
    dfields = []
    for i, (p, fl) in enumerate(members):
        d = {k: torch.from_numpy(inputs.f32(fl[k]).ravel()).to(dev) for k in ("K", "phi", "P0", "S0")}
        dfields.append(d)
        b.set_fields(i, d["K"], d["phi"])
        b.set_state(i, d["P0"], d["S0"])
    t_tune = time.perf_counter()
    nt = b.autotune(sweeps=5)
    t_tune = time.perf_counter() - t_tune
    tilings = {}
    for i, (p, _) in enumerate(members):
        tilings.setdefault(f"{p['shape'][0]}x{p['shape'][1]}", b.tiling(i))
    print(f"autotuned ensemble sweep: {nt} threads per block; blocked tilings (waves, rows per wave, "
          f"sweeps per launch) {tilings}, {t_tune:.1f} s", file=sys.stderr, flush=True)
    b.step(a.warmup, -1.0, it)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(a.steps, -1.0, it)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    mlups_batch = cells * a.steps * (it + 1) / t_batch / 1e6
    print(f"batched: {a.steps} steps in {t_batch:.3f} s", file=sys.stderr, flush=True)
    b.close()
    # the same members, one after another
    t_seq = 0.0
    for i, (p, fl) in enumerate(members):
        s = lbtp.from_problem(p, m=a.m, storage=a.storage)
        d = dfields[i]
        s.set_fields(d["K"], d["phi"])
        s.set_state(d["P0"], d["S0"])
        s.step(a.warmup, -1.0, it)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(a.steps, -1.0, it)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        s.close()
        del s
    mlups_seq = cells * a.steps * (it + 1) / t_seq / 1e6
    print(f"sequential: {t_seq:.3f} s", file=sys.stderr, flush=True)
    out = {
        "metric": "MLUPS (both lattices) + s/coupled step vs plain FP32 at residual 1e-8",
        "value": round(mlups_batch, 1), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(t_batch / a.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if a.storage == "fp32" else f"f32 math, {a.storage} storage",
        "data": "synthetic",
        "config": {"workload": f"ensemble of {len(members)} 2-D injection realisations, sides 128-1024, "
                               f"sigma_lnK in [0.5, 2], {it} pressure iterations per coupled step",
                   "cells": cells, "storage": a.storage, "threads_per_block": nt,
                   "blocked_tilings": {k: {"waves": v[0], "rows_per_wave": v[1], "sweeps_per_launch": v[2]}
                                       for k, v in tilings.items()},
                   "autotune_s": round(t_tune, 2)},
        "sequential_mlups": round(mlups_seq, 1), "batched_over_sequential": round(t_seq / t_batch, 3),
    }
    print(json.dumps(out), flush=True)


def ensemble_leg(storage, m, tol, n_members=32, steps=4, sizes=(128, 256)):
    """Batching against plain FP32 at the same residual: n_members 2-D
    injection realisations (sides from `sizes`, sigma_lnK in [0.5, 2]) for
    `steps` coupled steps to r <= tol (the first solve cold), advanced together
    (lbtp_batch, per-member stopping) and one after another through single
    contexts.  The iteration counts of the two runs must agree."""
    import torch
    from paper_1808_07554_amd import inputs, lbtp
    dev = torch.device("cuda", 0)
    members = inputs.ensemble(n_members, sizes=sizes)
    dfields = [{k: torch.from_numpy(inputs.f32(fl[k]).ravel()).to(dev) for k in ("K", "phi", "P0", "S0")}
               for _, fl in members]
    cells = np.array([p["shape"][0] * p["shape"][1] for p, _ in members], dtype=np.float64)
    b = lbtp.Batch([p for p, _ in members], m=m, storage=storage)
    for i, d in enumerate(dfields):
        b.set_fields(i, d["K"], d["phi"])
        b.set_state(i, d["P0"], d["S0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_b, _ = b.step(steps, tol, 10_000_000)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    t_seq, its_s = 0.0, []
    for i, (p, _) in enumerate(members):
        s = lbtp.from_problem(p, m=m, storage=storage)
        d = dfields[i]
        s.set_fields(d["K"], d["phi"])
        s.set_state(d["P0"], d["S0"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, _ = s.step(steps, tol, 10_000_000)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        its_s.append(list(its))
        s.close()
    its_s = np.array(its_s, dtype=np.int64).T   # [steps, members]
    updates = float(np.sum(cells * (its_b.sum(axis=0) + steps)))
    return {"members": n_members, "sides": list(sizes), "coupled_steps": steps, "tol": tol,
            "batched_mlups": round(updates / t_batch / 1e6, 1),
            "sequential_mlups": round(updates / t_seq / 1e6, 1),
            "batched_over_sequential": round(t_seq / t_batch, 3),
            "iterations_equal": bool(np.array_equal(its_b, its_s)),
            "iterations_total": int(its_b.sum())}


def warmstart_leg(train_pairs=2048, train_size=64, train_steps=1000, eval_fields=32, eval_size=256):
    """The learned start against the plain linear start at the same residual:
    a network trained briefly on the GPU (its own kernels) on solver-generated
    pairs, then held-out fields solved to r <= 1e-8 from both starts (wall
    time of the network start includes inference)."""
    from paper_1808_07554_amd import lbtp, warmstart as ws
    t0 = time.perf_counter()
    lnK, S, P, _ = ws.training_set(train_pairs, train_size, 1_000_000, factors=(1, 2, 4), log=False)
    t_data = time.perf_counter() - t0
    net = lbtp.WarmStartNet(32, 4, 3.2)
    net.set_params(ws.init_params(32, 4, seed=0))
    t0 = time.perf_counter()
    ws.train(net, lnK, S, P, train_steps, 32, 1e-3, log_every=0, weight=ws.relative_weights(P))
    t_train = time.perf_counter() - t0
    eK, eS, ephi = ws.fields(eval_fields, eval_size, 6_500_000)
    r = ws.evaluate(net, eK, eS, ephi, eval_size // train_size, starts=("linear", "network"))
    net.close()
    cold, warm = r["starts"]["linear"], r["starts"]["network"]
    return {"train_pairs": train_pairs, "train_size": train_size, "train_steps": train_steps,
            "data_s": round(t_data, 1), "train_s": round(t_train, 1),
            "eval_fields": eval_fields, "eval_size": eval_size, "tol": 1e-8,
            "linear_iterations_mean": round(cold["iterations_mean"], 1),
            "network_iterations_mean": round(warm["iterations_mean"], 1),
            "iteration_ratio": round(warm["iteration_ratio"], 3),
            "wall_ratio_with_inference": round(warm["wall_ratio"], 3),
            "fields_improved": round(warm["fewer_iterations_fraction"], 3)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1808_07554_amd import inputs, lbtp

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.workload == "ensemble":
        ensemble_bench(a)
        return
    if a.workload == "injection3d":
        params, fl = inputs.injection_3d(512 if a.n == 4096 else a.n)
        ncell = int(np.prod(params["shape"]))
    elif a.workload == "five-spot":
        if a.n == 4096:
            a.n = 96
        params, fl = inputs.five_spot(a.n)
        ncell = a.n * a.n
    else:
        params, fl = inputs.injection_2d(a.n)
        if a.lattice == "D2Q9":
            # eq. 3-4 needs max(phi)/2 <= beta <= 2 min(phi): phi in [0.15, 0.3] -> beta 0.2
            params = dict(params, lattice="D2Q9", beta=0.2)
        ncell = a.n * a.n
    def make_solver(storage):
        K = torch.from_numpy(inputs.f32(fl["K"]).ravel()).to(dev)
        phi = torch.from_numpy(inputs.f32(fl["phi"]).ravel()).to(dev)
        P0 = torch.from_numpy(inputs.f32(fl["P0"]).ravel()).to(dev)
        S0 = torch.from_numpy(inputs.f32(fl["S0"]).ravel()).to(dev)
        solver = lbtp.from_problem(params, m=a.m, storage=storage, sweep_block=a.sweep_block)
        solver.set_fields(K, phi)
        solver.set_state(P0, S0)
        del K, phi, P0, S0
        torch.cuda.synchronize()
        return solver

    def coupled_step(solver, progress=False):
        """One coupled step: coefficients, pressure solve to tol, saturation step.
        The solve runs in calls of 64k iterations so a long (cold) solve reports
        progress; each call continues the same iteration (checks stay on
        multiples of m)."""
        solver.update_coefficients()
        total, t0 = 0, time.perf_counter()
        while True:
            k, r, st = solver.pressure_solve(a.tol, min(65536, a.max_iters - total))
            total += k
            if progress:
                print(f"  cold solve: {total} iterations, r = {r:.3e}, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
            if st == lbtp.OK or total >= a.max_iters:
                break
            if st < 0:
                raise RuntimeError(f"pressure solve failed: {st}")
        solver.saturation_step()
        return total

    def run_leg(solver, label):
        """W warm-up coupled steps (the first is the cold solve), then K timed
        steps between two synchronisations."""
        warm, t_cold = [], None
        for w in range(a.warmup):
            t0 = time.perf_counter()
            warm.append(coupled_step(solver, progress=(w == 0)))
            torch.cuda.synchronize()
            if w == 0:
                t_cold = time.perf_counter() - t0
            print(f"{label} warmup step {w}: {warm[-1]} iterations, {time.perf_counter() - t0:.3f} s",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for k in range(a.steps):
            its.append(coupled_step(solver))
            if (k + 1) % 10 == 0:
                print(f"{label} timed step {k + 1}: {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t0
        print(f"{label} timed: {a.steps} steps in {t_run:.3f} s, iterations {sum(its)}", file=sys.stderr, flush=True)
        return dict(warm=warm, t_cold=t_cold, its=its, t_run=t_run,
                    mlups=ncell * (sum(its) + a.steps) / t_run / 1e6)

    s = make_solver(a.storage)
    main_leg = run_leg(s, a.storage)
    warm_its, t_cold, its_all, t_run = main_leg["warm"], main_leg["t_cold"], main_leg["its"], main_leg["t_run"]
    f_updates = sum(its_all)
    mlups = main_leg["mlups"]

    # the rest of the configured 5000 coupled steps (2-D injection), timed on
    # their own: the timed window above covers only the early steps after the
    # cold solve, when the front is young and the solves are longest
    config_steps = 5000 if (a.workload == "injection2d" and not a.no_tail) else 0
    tail = None
    done = a.warmup + a.steps
    if config_steps > done:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tail_its = []
        for k in range(config_steps - done):
            tail_its.append(coupled_step(s))
            if (k + 1) % 1000 == 0:
                print(f"tail step {done + k + 1}: {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_tail = time.perf_counter() - t0
        warm_all = warm_its[1:] + its_all + tail_its
        t_warm_all = t_run + t_tail            # warm-up steps 2..W are not timed; steps W+1..5000 are
        n_warm_timed = len(its_all) + len(tail_its)
        tail = {"steps": f"{a.warmup + 1}..{config_steps}", "s_per_coupled_step": t_warm_all / n_warm_timed,
                "iterations_per_step_mean": (sum(its_all) + sum(tail_its)) / n_warm_timed,
                "mlups": round(ncell * (sum(its_all) + sum(tail_its) + n_warm_timed) / t_warm_all / 1e6, 1),
                "iterations_per_step_percentiles": {q: int(np.percentile(warm_all, q)) for q in (50, 90, 99)}}
        print(f"steps {a.warmup + 1}..{config_steps}: {t_warm_all:.2f} s", file=sys.stderr, flush=True)

    # dominant kernel: a burst of back-to-back launches of the plain pressure
    # sweep (lbtp_probe_sweeps), HIP events on the solver's stream
    stream = torch.cuda.current_stream()
    s.update_coefficients()
    s.pressure_solve(-1.0, 20)
    s.probe_sweeps(2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    H = s.probe_sweeps(a.burst)
    e1.record(stream)
    torch.cuda.synchronize()
    launch_s = e0.elapsed_time(e1) / 1e3 / a.burst
    sweep_s = launch_s / H
    # saturation side (after the timed region; advances the state further)
    nsat = 10
    e0.record(stream)
    for _ in range(nsat):
        s.update_coefficients()
    e1.record(stream)
    torch.cuda.synchronize()
    moments_s = e0.elapsed_time(e1) / 1e3 / nsat
    gstep_s = 0.0
    for _ in range(nsat):      # a saturation step needs a pressure solve after the coefficients
        s.update_coefficients()
        s.pressure_solve(-1.0, 1)
        e0.record(stream)
        s.saturation_step()
        e1.record(stream)
        torch.cuda.synchronize()
        gstep_s += e0.elapsed_time(e1) / 1e3 / nsat
    alg_bytes = f_sweep_bytes(params["lattice"], a.storage) * ncell
    traffic = (measured_traffic(a.storage, params["lattice"])
               if (a.workload in ("injection2d", "injection3d") and a.n == 4096 and H > 1) else None)
    kname = sweep_kernel_name(a.storage, 3 if a.workload == "injection3d" else 2, params["lattice"], H)
    if H > 1:
        flops = BLOCK_FLOPS_PER_NODE_SWEEP[params["lattice"]] * ncell * H
        achieved = flops / launch_s / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(ALU_PEAK_TFLOPS, 2),
                    "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": traffic,
                    "kernel": f"{kname} ({H} plain pressure sweeps per launch)",
                    "avg_launch_us": round(launch_s * 1e6, 2), "flops_per_launch": flops,
                    "method_flops_per_node_sweep": BLOCK_FLOPS_PER_NODE_SWEEP[params["lattice"]],
                    # temporal blocking: H sweeps per HBM round trip of the populations
                    "blocking_factor": H,
                    "one_pass_bytes_per_launch": alg_bytes,
                    "one_pass_GBps": round(alg_bytes / launch_s / 1e9, 1),
                    "counter_GBps": round(traffic / launch_s / 1e9, 1) if traffic else None,
                    "counter_over_one_pass": round(traffic / alg_bytes, 3) if traffic else None,
                    # what H one-sweep launches would have to stream per second for the
                    # same work; above the HBM peak because the H sweeps share one pass
                    "sweep_equivalent_GBps": round(alg_bytes * H / launch_s / 1e9, 1)}
    else:
        achieved = alg_bytes / sweep_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": kname + " (plain pressure sweep)", "avg_launch_us": round(launch_s * 1e6, 2),
                    "bytes_per_launch": alg_bytes}

    out = {
        "metric": "MLUPS (both lattices) + s/coupled step vs plain FP32 at residual 1e-8",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(t_run / a.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.storage == "fp32" else f"f32 math, {a.storage} storage",
        "data": "synthetic",
        "config": {"workload": (f"heterogeneous injection 2-D {a.n}x{a.n} (log-normal K sigma 1, corr. length 16)"
                                if a.workload == "injection2d" else
                                f"five-spot (Section 4.3, Table 1 values) {a.n}x{a.n}, dt = {params['dt']:.4g}"
                                if a.workload == "five-spot" else
                                "heterogeneous injection 3-D %dx%dx%d (log-normal K sigma 1.5, corr. length 8)"
                                % tuple(params["shape"])),
                   "lattice": params["lattice"], "storage": a.storage, "tol": a.tol, "residual_stride": a.m,
                   "cells": ncell},
        "s_per_coupled_step": t_run / a.steps,
        "iterations_per_step_mean": f_updates / a.steps,
        "iterations_per_step_max": max(its_all),
        "iterations_per_step_percentiles": {q: int(np.percentile(its_all, q)) for q in (50, 90, 99)},
        "f_sweep_mlups": round(ncell / sweep_s / 1e6, 1),
        "g_step_mlups": round(ncell / gstep_s / 1e6, 1),
        "moments_us": round(moments_s * 1e6, 2),
        "g_step_us": round(gstep_s * 1e6, 2),
        "whole_job_s": (t_cold or 0.0) + t_run,
        "cold_first_step_s": t_cold,
        "cold_first_step_iterations": warm_its[0] if warm_its else None,
        "f_sweep_us": round(sweep_s * 1e6, 2),
        "roofline": roofline,
    }
    if tail is not None:
        out["config_mean"] = tail
    if a.workload == "injection2d" and a.storage == "fp32" and not a.no_legs:
        # the reduced-precision storage forms on the same workload and tolerance
        s.close()
        del s
        torch.cuda.synchronize()
        legs = {}
        for st in ("fp16", "bf16"):
            sl = make_solver(st)
            leg = run_leg(sl, st)
            sl.close()
            del sl
            torch.cuda.synchronize()
            legs[st] = {"value": round(leg["mlups"], 1), "unit": "MLUPS",
                        "s_per_coupled_step": leg["t_run"] / a.steps,
                        "iterations_per_step_mean": sum(leg["its"]) / a.steps,
                        "cold_first_step_s": leg["t_cold"],
                        "cold_first_step_iterations": leg["warm"][0] if leg["warm"] else None,
                        "mlups_over_fp32": round(leg["mlups"] / mlups, 3),
                        "step_time_fp32_over_this": round(t_run / leg["t_run"], 3),
                        "cold_solve_fp32_over_this": round(t_cold / leg["t_cold"], 3) if t_cold else None}
        out["storage_legs"] = legs
        # batching and the learned start against plain FP32 at the same residual
        t0 = time.perf_counter()
        out["ensemble_leg"] = ensemble_leg("fp32", a.m, a.tol)
        print(f"ensemble leg: {out['ensemble_leg']['batched_over_sequential']}x batched over sequential, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        out["warmstart_leg"] = warmstart_leg()
        print(f"warm-start leg: {out['warmstart_leg']['iteration_ratio']}x fewer iterations, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if not a.no_cpu and a.workload == "injection2d":
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
