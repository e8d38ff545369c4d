"""The largest 2-D problem the 32-bit cell indexing admits on D2Q5
(20480 x 20960 nodes: 5 x 429 260 800 < 2^31, about 45 GB of device
memory), in the benchmark's launch configuration (blocked sweeps, m = 64):
sampled nodes against the oracle on crops, as at the benchmark size.  The
fields are smooth and separable, so that they are cheap to build at this
size and the crops see exactly the values the GPU gets (float32 products
and sums of float32 factors)."""
import time

import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.test_gpu_fullsize import _check_samples, _samples

pytestmark = pytest.mark.gpu

NX, NY = 20480, 20960


def _fields(nx, ny):
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    params, _ = inputs.injection_problem((8, 8), 1.0, 4.0, 1, 2)
    params = dict(params, shape=(nx, ny, 1))
    K0 = np.float32(params["mu_n"] / 6.0)
    kx = np.exp(0.5 * np.sin(2 * np.pi * x / 97.0)).astype(np.float32)
    ky = np.exp(0.5 * np.cos(2 * np.pi * y / 61.0)).astype(np.float32)
    K = np.multiply.outer(ky, kx * K0)                                   # float32
    px = (0.03 * np.sin(2 * np.pi * x / 53.0)).astype(np.float32)
    py = (0.22 + 0.03 * np.cos(2 * np.pi * y / 41.0)).astype(np.float32)
    phi = np.add.outer(py, px)                                            # float32
    P0 = np.broadcast_to(((1.0 - (x + 0.5) / nx)).astype(np.float32), (ny, nx)).copy()
    S0 = np.zeros((ny, nx), np.float32)
    fl = {k: v.reshape(1, ny, nx) for k, v in dict(K=K, phi=phi, P0=P0, S0=S0).items()}
    return params, fl


def test_largest_2d_problem_sampled_parity():
    assert 5 * NX * NY < 2 ** 31
    t0 = time.perf_counter()
    params, fl = _fields(NX, NY)
    print(f"fields built in {time.perf_counter() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(29)
    worst = _check_samples(params, fl, _samples((NX, NY), rng, 3), "fp32")
    print(f"done in {time.perf_counter() - t0:.1f} s", flush=True)
    for k, v in worst.items():
        assert v <= 1e-5, (k, v)
