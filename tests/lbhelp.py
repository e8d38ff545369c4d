"""Shared test helpers: build the oracle and the GPU solver from one plain
parameter dict, compare fields.  (Test code: may import both sides.)"""
import numpy as np

import oracle
from paper_1808_07554_amd import inputs


def oracle_solver(params, m=1, dtype=np.float64):
    return oracle.Solver(params["lattice"], params["shape"], beta=params["beta"], Ds=params["Ds"],
                         coef=oracle.QuadraticKr(params["mu_w"], params["mu_n"]),
                         bc_f=params["bc_f"], bc_g=params["bc_g"], dx=params.get("dx", 1.0),
                         dt=params.get("dt", 1.0), m=m, dtype=dtype, cap_B=params.get("cap_B", 0.0),
                         collision=params.get("collision"))


def gpu_solver(params, m=64, **kw):
    from paper_1808_07554_amd import lbtp
    return lbtp.from_problem(params, m=m, **kw)


def f32(a):
    """float32-rounded copy as float64 (what both sides receive)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel_l2(ref, got):
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    den = np.sqrt(np.sum(ref * ref))
    return float(np.sqrt(np.sum((ref - got) ** 2)) / (den if den > 0 else 1.0))


def mean_free(a):
    a = np.asarray(a, dtype=np.float64)
    return a - a.mean()


def smooth_state(fshape, seed):
    """A smooth random S in (0.1, 0.9) and a pressure ramp with a smooth bump (float64)."""
    nz, ny, nx = fshape
    ell = max(2.0, min(nx, ny) / 6)
    z = inputs.gaussian_random_field(fshape if nz > 1 else (ny, nx), ell, seed).reshape(fshape)
    S = 0.5 + 0.3 * np.tanh(z)
    x = (np.arange(nx) + 0.5) / nx
    P = np.broadcast_to(1.0 - x, fshape) + 0.05 * np.tanh(z)
    return np.ascontiguousarray(P), S
