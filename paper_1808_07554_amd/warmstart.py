"""Learned warm start of the pressure iteration: training data from the
solver, training with the network's own kernels, and evaluation.

The network (include/lbtp_nn.h) maps (lnK, S, wall proximity) to an initial
pressure.  It is trained on one grid size and applied to an n x n grid on the
grid coarsened to that size, so the training pairs are drawn the way the
network sees them (training_set): seeded heterogeneous fields (log-normal K,
saturation S = logistic of a Gaussian random field) of the evaluation
statistics on grids f times larger, block-averaged by f, for a mix of
factors f, labelled with the block average of the fine problem's pressure.
The lattice Boltzmann solver itself produces the labels, solving every fine
problem to the stopping tolerance from the linear profile, many realisations
at a time with the ensemble API.  The
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


def _sample(n, seed, sigma, ell, coarse=1):
    """One seeded realisation at n x n, block-averaged by `coarse`:
    lnK = sigma * GRF(ell), S = logistic(1.5 * GRF(ell))."""
    base = 4 * seed
    lnK = sigma * inputs.gaussian_random_field((n, n), ell, base)
    S = 1.0 / (1.0 + np.exp(-1.5 * inputs.gaussian_random_field((n, n), ell, base + 1)))
    if coarse > 1:
        m = n // coarse
        lnK = lnK.reshape(m, coarse, m, coarse).mean(axis=(1, 3))
        S = S.reshape(m, coarse, m, coarse).mean(axis=(1, 3))
    return lnK, S


def fields(count, n, seed0, sigma=(0.5, 2.0), ell=(4.0, 16.0)):
    """Seeded inputs: lnK (sigma_lnK, correlation length drawn per sample),
    S = logistic(GRF) in (0, 1), phi ~ U[0.15, 0.3].  float32 [count, n, n]."""
    lnK = np.empty((count, n, n), np.float32)
    S = np.empty((count, n, n), np.float32)
    phi = np.empty((count, n, n), np.float32)
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        lnK[j], S[j] = _sample(n, seed0 + j, rng.uniform(*sigma), rng.uniform(*ell))
        phi[j] = inputs.uniform_field((n, n), 0.15, 0.3, 4 * (seed0 + j) + 2)
    return lnK, S, phi


def training_set(count, size, seed0, factors=(1, 2, 4, 8, 16), sigma=(0.5, 2.0), ell=(4.0, 16.0), chunk=512,
                 tol=1e-8, m=64, threads=8, log=True):
    """Training pairs on a size x size grid, as the network sees them when it
    runs on a grid coarsened by f: inputs are fields with the evaluation
    statistics on a grid f times finer, block-averaged by f, and the label is
    the block average of that fine problem's converged pressure (not the
    solution of the coarse problem, which misses the fine structure's effect
    on the long-wavelength modes).  Fine grids are capped at 4 size: a field
    of (f size)^2 with correlation length l averaged by f has the statistics
    of a (c size)^2 field with length c l / f averaged by c (only block /
    length matters), and the Darcy pressure with fixed end pressures does not
    depend on the length scale.  Returns lnK, S, P [count, size, size]
    float32 and the factor of every sample."""
    from concurrent.futures import ThreadPoolExecutor
    spec = []
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        f = int(factors[rng.integers(len(factors))])
        spec.append((seed0 + j, f, rng.uniform(*sigma), rng.uniform(*ell)))
    lnK = np.empty((count, size, size), np.float32)
    S = np.empty_like(lnK)
    P = np.empty_like(lnK)
    fac = np.array([sp[1] for sp in spec])
    csz = np.minimum(fac, 4)
    t0 = time.perf_counter()
    done = 0
    with ThreadPoolExecutor(threads) as ex:
        for c in sorted(set(csz.tolist())):
            idx = np.nonzero(csz == c)[0]
            n = c * size

            def make(j):
                seed, f, sg, l = spec[j]
                a, b = _sample(n, seed, sg, l * c / f)
                return a, b, inputs.uniform_field((n, n), 0.15, 0.3, 4 * seed + 2)
            for a in range(0, idx.size, chunk):
                part = idx[a:a + chunk]
                got = list(ex.map(make, part))
                fK = np.stack([g[0] for g in got]).astype(np.float32)
                fS = np.stack([g[1] for g in got]).astype(np.float32)
                fphi = np.stack([g[2] for g in got]).astype(np.float32)
                fP, _, _ = solve(fK, fS, fphi, None, tol, m)
                lnK[part] = _block_mean(fK, c)
                S[part] = _block_mean(fS, c)
                P[part] = _block_mean(fP.astype(np.float64), c)
                done += part.size
                if log:
                    print(f"  training pairs {done} / {count} (fine grid {n}^2, {time.perf_counter() - t0:.0f} s)",
                          file=sys.stderr, flush=True)
    return lnK, S, P, fac


def relative_weights(P):
    """Per-sample loss weights proportional to 1 / mean((P - linear profile)^2),
    normalised to mean 1: every sample counts by its relative error, so the
    small deviations of strongly coarsened fields are learned as well."""
    w = P.shape[-1]
    D = P - (1.0 - (np.arange(w) + 0.5) / w)
    inv = 1.0 / np.maximum(np.mean(D.astype(np.float64) ** 2, axis=(1, 2)), 1e-12)
    return (inv / inv.mean()).astype(np.float32)


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


def solve_chunked(lnK, S, phi, chunk=1024, P0=None, **kw):
    out, its, t = [], [], 0.0
    for a in range(0, lnK.shape[0], chunk):
        P, k, dt = solve(lnK[a:a + chunk], S[a:a + chunk], phi[a:a + chunk],
                         None if P0 is None else P0[a:a + chunk], **kw)
        out.append(P)
        its.append(k)
        t += dt
        print(f"  solved {a + P.shape[0]} / {lnK.shape[0]} fields ({dt:.1f} s)", file=sys.stderr, flush=True)
    return np.concatenate(out), np.concatenate(its), t


def train(net, lnK, S, P, steps, batch=32, lr=1e-3, seed=0, log_every=100, weight=None):
    """Adam on minibatches drawn with a seeded permutation; cosine-decayed lr;
    optional per-sample loss weights."""
    import torch
    rng = np.random.default_rng(seed)
    n = lnK.shape[0]
    dK = torch.from_numpy(lnK).cuda()
    dS = torch.from_numpy(S).cuda()
    dP = torch.from_numpy(P).cuda()
    dW = None if weight is None else torch.from_numpy(np.asarray(weight, np.float32)).cuda()
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
        losses.append(net.train_step(dK[idx], dS[idx], dP[idx], max(cur, lr * 1e-2),
                                     None if dW is None else dW[idx]))
        if log_every and (it + 1) % log_every == 0:
            print(f"  train step {it + 1}: loss {np.mean(losses[-log_every:]):.3e}", file=sys.stderr, flush=True)
    return losses


def _block_mean(x, f):
    n, h, w = x.shape
    return x.reshape(n, h // f, f, w // f, f).mean(axis=(2, 4))


def _refine_deviation(Pc, f):
    """Fine pressure from a coarse one: its deviation from the coarse linear
    profile, interpolated bilinearly to the fine node centres (edge values
    beyond the outer centres), plus the fine linear profile."""
    n, h, w = Pc.shape
    D = Pc - (1.0 - (np.arange(w) + 0.5) / w)

    def weights(m):
        u = np.clip((np.arange(m * f) + 0.5) / f - 0.5, 0, m - 1)
        i = np.minimum(np.floor(u).astype(int), m - 2) if m > 1 else np.zeros(m * f, int)
        return i, np.minimum(i + 1, m - 1), u - i
    y0, y1, ty = weights(h)
    x0, x1, tx = weights(w)
    R = D[:, y0, :] * (1 - ty)[None, :, None] + D[:, y1, :] * ty[None, :, None]
    R = R[:, :, x0] * (1 - tx) + R[:, :, x1] * tx
    return (1.0 - (np.arange(w * f) + 0.5) / (w * f)) + R


def evaluate(net, lnK, S, phi, factor=1, tol=1e-8, m=64, starts=("linear", "zero", "network", "coarse_solve"),
             chunk=32):
    """Solve the same fields to the same tolerance from several initial
    pressures and report iterations and wall time for each:
      linear        the linear profile between the Dirichlet walls (cold start)
      zero          P0 = 0
      network       the network's prediction (on the grid coarsened by factor)
      coarse_solve  the solver's own solution of the problem coarsened by
                    factor, refined like the network's output (a non-learned
                    coarse-grid start)
      ceiling       the block average of the converged pressure (from the
                    linear start), refined the same way: what a perfect
                    coarse-grid predictor would give
    Times include preparing the start (inference, the coarse solve).  Every
    start solves the fields in the same batches of `chunk` fields."""
    import torch
    count, n, _ = lnK.shape
    out = dict(fields=int(count), size=int(n), factor=int(factor))
    res = {}
    P_conv = None
    for st in starts:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if st == "linear":
            P0 = None
        elif st == "zero":
            P0 = np.zeros_like(lnK)
        elif st == "network":
            P0 = np.concatenate([net.predict(lnK[a:a + 16], S[a:a + 16], factor).cpu().numpy()
                                 for a in range(0, count, 16)])
        elif st == "coarse_solve":
            if factor == 1:
                continue
            Pc, _, _ = solve(_block_mean(lnK, factor), _block_mean(S, factor), _block_mean(phi, factor), None, tol, m)
            P0 = _refine_deviation(Pc.astype(np.float64), factor).astype(np.float32)
        elif st == "ceiling":
            Pc = _block_mean(P_conv.astype(np.float64), factor)
            P0 = _refine_deviation(Pc, factor).astype(np.float32) if factor > 1 else P_conv
        else:
            raise ValueError(st)
        torch.cuda.synchronize()
        t_prep = time.perf_counter() - t0
        Pk, its, t = solve_chunked(lnK, S, phi, chunk, P0=P0, tol=tol, m=m)
        if st == "linear":
            P_conv = Pk
        res[st] = dict(iterations_mean=float(its.mean()), iterations_median=float(np.median(its)),
                       solve_s=t, prepare_s=t_prep, its=its)
        print(f"  {n}^2 x {count}: {st} start {its.mean():.0f} iterations, {t + t_prep:.2f} s", file=sys.stderr,
              flush=True)
    cold = res["linear"]
    for st, r in res.items():
        if st != "linear":
            r["iteration_ratio"] = cold["iterations_mean"] / max(r["iterations_mean"], 1.0)
            r["wall_ratio"] = (cold["solve_s"] + cold["prepare_s"]) / (r["solve_s"] + r["prepare_s"])
            r["fewer_iterations_fraction"] = float(np.mean(r["its"] < cold["its"]))
    for r in res.values():
        del r["its"]
    out["starts"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-fields", type=int, default=20000)
    ap.add_argument("--train-size", type=int, default=64)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--scale", type=float, default=3.2, help="output scale per node (P - ramp = scale / W * net)")
    ap.add_argument("--eval", default="64:500,256:64,1024:16", help="size:count,...")
    ap.add_argument("--starts", default="linear,zero,network,coarse_solve,ceiling",
                    help="initial pressures to compare (linear first)")
    ap.add_argument("--no-weights", action="store_true", help="plain (unweighted) mean squared error")
    ap.add_argument("--load", default=None, help="start from these weights (.npy) instead of training from scratch")
    ap.add_argument("--out", default=None, help="write the report (JSON) and weights (.npy) with this prefix")
    ap.add_argument("--eval-seed", type=int, default=6_000_000,
                    help="seed of the first held-out field (item j of --eval starts 100 000 j later)")
    a = ap.parse_args()
    rep = {}
    net = lbtp.WarmStartNet(32, 4, a.scale)
    if a.load:
        with open(a.load, "rb") as f:        # a .npy file under any name
            net.set_params(np.load(f).astype(np.float32))
    else:
        t0 = time.perf_counter()
        lnK, S, P, fac = training_set(a.train_fields, a.train_size, 1_000_000)
        rep["training_data"] = dict(fields=a.train_fields, size=a.train_size, seconds=time.perf_counter() - t0,
                                    factors={int(f): int((fac == f).sum()) for f in np.unique(fac)})
        print(json.dumps(rep["training_data"]), file=sys.stderr, flush=True)
        net.set_params(init_params(32, 4, seed=0))
        t0 = time.perf_counter()
        wts = None if a.no_weights else relative_weights(P)
        losses = train(net, lnK, S, P, a.steps, a.batch, a.lr, weight=wts)
        rep["training"] = dict(steps=a.steps, batch=a.batch, seconds=time.perf_counter() - t0,
                               weighted=wts is not None,
                               loss_first=float(np.mean(losses[:50])), loss_last=float(np.mean(losses[-50:])))
        print(json.dumps(rep["training"]), file=sys.stderr, flush=True)
        if a.out:
            np.save(a.out + "_weights.npy", net.get_params().cpu().numpy())
    rep["eval"] = []
    for j, item in enumerate(a.eval.split(",")):
        size, count = (int(v) for v in item.split(":"))
        eK, eS, ephi = fields(count, size, a.eval_seed + 100_000 * j)
        r = evaluate(net, eK, eS, ephi, max(1, size // a.train_size), starts=a.starts.split(","))
        rep["eval"].append(r)
        print(json.dumps(r), file=sys.stderr, flush=True)
        if a.out:
            with open(a.out + ".json", "w") as f:
                json.dump(rep, f, indent=1)
    print(json.dumps(rep), flush=True)


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
