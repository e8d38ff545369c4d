"""Per-field errors of the 3-D injection workload against the float64 oracle,
per storage format (test infrastructure; not collected by pytest).

The 3-D injection recipe (log-normal K with sigma 1.5 and correlation length
8, phi uniform in [0.15, 0.3], x the flow axis, walled y and z faces) at 64^3:
a cold pressure solve to r <= tol from the linear profile, then coupled steps
(coefficients, pressure solve to tol, saturation step).

    python -m tests.c3_field_errors oracle OUT.npz [--n 64] [--steps 20]
runs the oracle and stores its pressure-iteration counts per step and its
P, u, S after the last solve (rewritten after every step, so a long run can
be cut short);
    python -m tests.c3_field_errors gpu REF.npz [--json OUT.json]
replays those iteration counts through the C ABI with float32, fp16 and bf16
storage and prints relative L2 and max errors (max |got - ref| / max |ref|)
of P, u (all components) and S."""
import argparse
import json
import sys
import time

import numpy as np

from paper_1808_07554_amd import inputs
from tests.lbhelp import f32, oracle_solver, rel_l2


def _problem(n):
    params, fl = inputs.injection_3d(n)
    return params, f32(fl["K"]), f32(fl["phi"]), f32(fl["P0"]), f32(fl["S0"])


def run_oracle(out, n, steps, tol, m):
    params, K, phi, P0, S0 = _problem(n)
    o = oracle_solver(params, m=m)
    o.set_fields(K, phi)
    o.set_state(P0, S0)
    its = []
    t0 = time.perf_counter()
    for s in range(steps + 1):
        o.update_coefficients()
        k, r, st = o.pressure_solve(tol, 10_000_000)
        its.append(int(k))
        print(f"oracle step {s}: {k} iterations, r = {r:.3e}, {time.perf_counter() - t0:.0f} s", flush=True)
        # the reference after the solve of every step (a long run can be cut)
        np.savez(out, n=n, its=np.array(its), tol=tol, m=m, P=o.pressure(), u=o.velocity(), S=o.saturation())
        if s < steps:
            o.saturation_step()


def _errors(ref, got):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    return rel_l2(ref, got), float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def run_gpu(ref_path, json_out):
    from paper_1808_07554_amd import lbtp  # noqa: F401  (the library under test)
    from tests.lbhelp import gpu_solver
    ref = np.load(ref_path)
    n, its, m = int(ref["n"]), [int(k) for k in ref["its"]], int(ref["m"])
    params, K, phi, P0, S0 = _problem(n)
    rows = {}
    for storage in ("fp32", "fp16", "bf16"):
        g = gpu_solver(params, m=m, storage=storage)
        g.set_fields(K, phi)
        g.set_state(P0, S0)
        for s, k in enumerate(its):
            g.update_coefficients()
            done = g.pressure_solve(-1.0, k)[0]
            assert done == k, (storage, s, done, k)
            if s < len(its) - 1:
                g.saturation_step()
        P = g.pressure().cpu().numpy().reshape(ref["P"].shape)
        u = g.velocity().cpu().numpy().reshape(ref["u"].shape[0], *ref["P"].shape)
        S = g.saturation().cpu().numpy().reshape(ref["S"].shape)
        g.close()
        rows[storage] = {"P": _errors(ref["P"], P), "u": _errors(ref["u"][: u.shape[0]], u), "S": _errors(ref["S"], S)}
        print(storage, {k: f"L2 {v[0]:.2e} max {v[1]:.2e}" for k, v in rows[storage].items()}, flush=True)
    warm = f", then {min(its[1:])}-{max(its[1:])}" if len(its) > 1 else ""
    lines = [f"{n}^3 D3Q7 injection, the cold solve and {len(its) - 1} coupled steps "
             f"(oracle iterations per solve: {its[0]} cold{warm}), replayed with the oracle's counts",
             "| storage | P L2 | P max | u L2 | u max | S L2 | S max |", "|---|---|---|---|---|---|---|"]
    for st, r in rows.items():
        lines.append(f"| {st} | " + " | ".join(f"{r[k][0]:.1e} | {r[k][1]:.1e}" for k in ("P", "u", "S")) + " |")
    print("\n".join(lines))
    if json_out:
        with open(json_out, "w") as f:
            json.dump({"its": its, "errors": rows}, f, indent=1)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["oracle", "gpu"])
    ap.add_argument("path")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--m", type=int, default=64)
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    if a.what == "oracle":
        run_oracle(a.path, a.n, a.steps, a.tol, a.m)
    else:
        run_gpu(a.path, a.json)
    sys.exit(0)
