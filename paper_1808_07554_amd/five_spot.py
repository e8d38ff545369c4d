"""The five-spot problem of Section 4.3 on the GPU path (D2Q9).

Inputs come from paper_1808_07554_amd.inputs.five_spot (Table 1 values, the
quarter pattern with wells as Dirichlet segments of the walls at opposite
corners, set link by link through lbtp_set_wall_types).  Each coupled step
solves the pressure lattice to the stopping rule and advances the
saturation lattice once, as in Section 3.

    python -m paper_1808_07554_amd.five_spot [--sizes 32 64 96] [--T 10]

prints the saturation and pressure along the diagonal from the injector to
the producer at time T for each lattice size and the largest differences
between successive sizes (the grid-independence study of Section 4.3).
"""
import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbtp


def make_solver(N, storage="fp32", m=64, **kw):
    """A Solver holding the N x N five-spot problem at t = 0."""
    params, fl = inputs.five_spot(N, **kw)
    s = lbtp.from_problem(params, m=m, storage=storage)
    s.set_fields(inputs.f32(fl["K"]).ravel(), inputs.f32(fl["phi"]).ravel())
    s.set_state(inputs.f32(fl["P0"]).ravel(), inputs.f32(fl["S0"]).ravel())
    return s, params


def coupled_step(s, tol, max_iters):
    """Coefficients at S^n, pressure solve to tol, saturation step; returns
    the pressure iterations."""
    s.update_coefficients()
    k, r, st = s.pressure_solve(tol, max_iters)
    if st < 0:
        raise RuntimeError(f"pressure solve failed with status {st} (r = {r})")
    s.saturation_step()
    return k


def diagonal(a):
    """Values at the nodes (i, i), injector to producer."""
    a = np.asarray(a).reshape(a.shape[-2], a.shape[-1])
    return np.diag(a).astype(np.float64)


def run(N, T=10.0, tol=1e-8, max_iters=1_000_000, storage="fp32", progress=None):
    """Advance the N x N five-spot problem to time T.  Returns a dict with the
    diagonal profiles of S and P at T, the step and iteration counts and the
    wall time on the GPU (inputs already resident)."""
    import torch
    s, params = make_solver(N, storage)
    nsteps = int(round(T / params["dt"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for n in range(nsteps):
        its.append(coupled_step(s, tol, max_iters))
        if progress and (n + 1) % progress == 0:
            print(f"  N={N}: step {n + 1}/{nsteps}, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    # the pressure and velocity at T: one more solve at S(T)
    s.update_coefficients()
    s.pressure_solve(tol, max_iters)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    S = s.saturation().cpu().numpy()
    P = s.pressure().cpu().numpy()
    mass, ledger = s.mass()
    s.close()
    return dict(N=N, T=T, steps=nsteps, dt=params["dt"], iterations=int(sum(its)), first_solve=its[0] if its else 0,
                seconds=wall, S_diag=diagonal(S), P_diag=diagonal(P), mass=mass, ledger=ledger)


def on_common_diagonal(res, n_pts=33):
    """Profiles of a run interpolated to n_pts equally spaced points of the
    diagonal's node range shared by all sizes (fraction 0..1 of x + y)."""
    N = res["N"]
    frac = (np.arange(N) + 0.5) / N
    q = np.linspace(0.1, 0.9, n_pts)
    return q, np.interp(q, frac, res["S_diag"]), np.interp(q, frac, res["P_diag"])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", type=int, nargs="+", default=[32, 64, 96])
    ap.add_argument("--T", type=float, default=10.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--json", help="write the profiles to this file")
    a = ap.parse_args(argv)
    results = []
    for N in a.sizes:
        r = run(N, a.T, a.tol, storage=a.storage, progress=2000)
        results.append(r)
        print(f"N={N}: {r['steps']} coupled steps, {r['iterations']} pressure iterations "
              f"(first solve {r['first_solve']}), {r['seconds']:.2f} s", flush=True)
    prof = [on_common_diagonal(r) for r in results]
    q = prof[0][0]
    print("x+y fraction  " + "  ".join(f"S(N={r['N']})  P(N={r['N']})" for r in results))
    for i in range(0, len(q), 4):
        print(f"{q[i]:.3f}        " + "  ".join(f"{p[1][i]:.4f}     {p[2][i]:.4f}   " for p in prof))
    for (r0, p0), (r1, p1) in zip(zip(results, prof), zip(results[1:], prof[1:])):
        print(f"N={r0['N']} vs N={r1['N']}: max |dS| {np.abs(p0[1] - p1[1]).max():.4f}, "
              f"max |dP| {np.abs(p0[2] - p1[2]).max():.4f}")
    if a.json:
        with open(a.json, "w") as f:
            json.dump([{k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in r.items()} for r in results],
                      f)


if __name__ == "__main__":
    main()
