"""Learned warm start of the pressure iteration: training data from the
solver, training with the network's own kernels, and evaluation.

The network (include/lbtp_nn.h) maps (lnK, S, x/L) to an initial pressure.
Training pairs come from the lattice Boltzmann solver itself: for seeded
heterogeneous fields (log-normal K, saturation S = logistic of a Gaussian
random field) the pressure is solved to the stopping tolerance from the
linear profile, many realisations at a time with the ensemble API.  The
evaluation solves held-out fields twice to the same tolerance, once from the
linear profile (cold) and once from the network's prediction (warm), and
reports pressure iterations and wall time (the warm time includes
inference).

    python -m paper_1808_07554_amd.warmstart --help
"""
import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbtp

MU_W, MU_N, BETA = 1.0, 5.0, 0.15
K0 = (1.0 / 3.0) * MU_N / 2
DS = BETA * (1.0 / 3.0) / 2


def problem(n):
    """2-D injection problem on an n x n grid (D2Q5, lattice units)."""
    return dict(lattice="D2Q5", shape=(n, n, 1), dx=1.0, dt=1.0, beta=BETA, Ds=DS, mu_w=MU_W, mu_n=MU_N,
                bc_f=[("abb", 1.0), ("abb", 0.0), ("bb",), ("bb",)],
                bc_g=[("abb", 1.0), ("outflow",), ("bb",), ("bb",)])


def fields(count, n, seed0, sigma=(0.5, 2.0), ell=(4.0, 16.0)):
    """Seeded inputs: lnK (sigma_lnK, correlation length drawn per sample),
    S = logistic(GRF) in (0, 1), phi ~ U[0.15, 0.3].  float32 [count, n, n]."""
    lnK = np.empty((count, n, n), np.float32)
    S = np.empty((count, n, n), np.float32)
    phi = np.empty((count, n, n), np.float32)
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        s = rng.uniform(*sigma)
        l = rng.uniform(*ell)
        base = 4 * (seed0 + j)
        lnK[j] = s * inputs.gaussian_random_field((n, n), l, base)
        S[j] = 1.0 / (1.0 + np.exp(-1.5 * inputs.gaussian_random_field((n, n), l, base + 1)))
        phi[j] = inputs.uniform_field((n, n), 0.15, 0.3, base + 2)
    return lnK, S, phi


def solve(lnK, S, phi, P0=None, tol=1e-8, m=64, max_iters=None, storage="fp32"):
    """Pressure of every field to r <= tol (one coupled step's solve, ensemble
    API).  P0: initial pressure [count, n, n] or None for the linear profile.
    Returns (P [count, n, n] float32 numpy, iterations per field, seconds)."""
    import torch
    count, n, _ = lnK.shape
    max_iters = max_iters or m * 100000
    b = lbtp.Batch([problem(n)] * count, m=m, storage=storage)
    ramp = np.broadcast_to((1.0 - (np.arange(n) + 0.5) / n).astype(np.float32), (n, n))
    dev = torch.device("cuda", 0)
    for j in range(count):
        K = torch.from_numpy(np.ascontiguousarray(K0 * np.exp(lnK[j]))).to(dev)
        b.set_fields(j, K.ravel(), torch.from_numpy(phi[j]).to(dev).ravel())
        p0 = ramp if P0 is None else P0[j]
        b.set_state(j, torch.from_numpy(np.ascontiguousarray(p0)).to(dev).ravel(),
                    torch.from_numpy(S[j]).to(dev).ravel())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, _ = b.step(1, tol, max_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    P = np.stack([b.pressure(j).cpu().numpy().reshape(n, n) for j in range(count)])
    b.close()
    return P, its[0], dt


def solve_chunked(lnK, S, phi, chunk=1024, **kw):
    out, its, t = [], [], 0.0
    for a in range(0, lnK.shape[0], chunk):
        P, k, dt = solve(lnK[a:a + chunk], S[a:a + chunk], phi[a:a + chunk], **kw)
        out.append(P)
        its.append(k)
        t += dt
        print(f"  solved {a + P.shape[0]} / {lnK.shape[0]} fields ({dt:.1f} s)", file=sys.stderr, flush=True)
    return np.concatenate(out), np.concatenate(its), t


def train(net, lnK, S, P, steps, batch=32, lr=1e-3, seed=0, log_every=100):
    """Adam on minibatches drawn with a seeded permutation; cosine-decayed lr."""
    import torch
    rng = np.random.default_rng(seed)
    n = lnK.shape[0]
    dK = torch.from_numpy(lnK).cuda()
    dS = torch.from_numpy(S).cuda()
    dP = torch.from_numpy(P).cuda()
    losses = []
    order = rng.permutation(n)
    pos = 0
    for it in range(steps):
        if pos + batch > n:
            order = rng.permutation(n)
            pos = 0
        idx = torch.from_numpy(order[pos:pos + batch]).cuda()
        pos += batch
        cur = lr * 0.5 * (1 + np.cos(np.pi * it / steps))
        losses.append(net.train_step(dK[idx], dS[idx], dP[idx], max(cur, lr * 1e-2)))
        if log_every and (it + 1) % log_every == 0:
            print(f"  train step {it + 1}: loss {np.mean(losses[-log_every:]):.3e}", file=sys.stderr, flush=True)
    return losses


def evaluate(net, lnK, S, phi, tol=1e-8, m=64):
    """Cold (linear profile) and warm (network) starts of the same fields."""
    import torch
    _, its_cold, t_cold = solve(lnK, S, phi, None, tol, m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P0 = np.concatenate([net.predict(lnK[a:a + 16], S[a:a + 16]).cpu().numpy() for a in range(0, lnK.shape[0], 16)])
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    _, its_warm, t_warm = solve(lnK, S, phi, P0, tol, m)
    return dict(fields=int(lnK.shape[0]), size=int(lnK.shape[1]), cold_iterations_mean=float(its_cold.mean()),
                warm_iterations_mean=float(its_warm.mean()),
                iteration_ratio=float(its_cold.mean() / max(its_warm.mean(), 1)),
                cold_s=t_cold, warm_s=t_warm + t_inf, inference_s=t_inf,
                wall_ratio=float(t_cold / (t_warm + t_inf)),
                warm_better_fraction=float(np.mean(its_warm < its_cold)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-fields", type=int, default=20000)
    ap.add_argument("--train-size", type=int, default=64)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--scale", type=float, default=3.2, help="output scale per node (P - ramp = scale / W * net)")
    ap.add_argument("--eval", default="64:500,256:64,1024:16", help="size:count,...")
    ap.add_argument("--load", default=None, help="start from these weights (.npy) instead of training from scratch")
    ap.add_argument("--out", default=None, help="write the report (JSON) and weights (.npy) with this prefix")
    a = ap.parse_args()
    rep = {}
    t0 = time.perf_counter()
    lnK, S, phi = fields(a.train_fields, a.train_size, 1_000_000)
    P, its, t_sol = solve_chunked(lnK, S, phi)
    rep["training_data"] = dict(fields=a.train_fields, size=a.train_size, solve_s=t_sol,
                                iterations_mean=float(its.mean()), generate_s=time.perf_counter() - t0)
    print(json.dumps(rep["training_data"]), file=sys.stderr, flush=True)
    net = lbtp.WarmStartNet(32, 4, a.scale)
    net.set_params(init_params(32, 4, seed=0))
    t0 = time.perf_counter()
    losses = train(net, lnK, S, P, a.steps, a.batch, a.lr)
    rep["training"] = dict(steps=a.steps, batch=a.batch, seconds=time.perf_counter() - t0,
                           loss_first=float(np.mean(losses[:50])), loss_last=float(np.mean(losses[-50:])))
    print(json.dumps(rep["training"]), file=sys.stderr, flush=True)
    rep["eval"] = []
    for j, item in enumerate(a.eval.split(",")):
        size, count = (int(v) for v in item.split(":"))
        eK, eS, ephi = fields(count, size, 6_000_000 + 100_000 * j)
        r = evaluate(net, eK, eS, ephi)
        rep["eval"].append(r)
        print(json.dumps(r), file=sys.stderr, flush=True)
    print(json.dumps(rep), flush=True)
    if a.out:
        with open(a.out + ".json", "w") as f:
            json.dump(rep, f, indent=1)
        np.save(a.out + "_weights.npy", net.get_params().cpu().numpy())


def init_params(base, levels, seed=0):
    """He-normal weights and zero biases, flat (the network's parameter layout)."""
    rng = np.random.default_rng(seed)
    c = [base * 2 ** l for l in range(levels)]
    io = []
    prev = 3
    for l in range(levels):
        io += [(prev, c[l], True), (c[l], c[l], True)]
        prev = c[l]
    for l in range(levels - 2, -1, -1):
        io += [(c[l + 1] + c[l], c[l], True), (c[l], c[l], True)]
    io.append((c[0], 1, False))
    parts = []
    for ci, co, relu in io:
        std = np.sqrt((2.0 if relu else 1.0) / (9 * ci))
        parts.append((rng.standard_normal((co, 3, 3, ci)) * std).ravel())
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


if __name__ == "__main__":
    main()
