"""Problems as large as the 32-bit cell indexing admits (Q x nodes < 2^31)
on each lattice, in the benchmark's launch configuration (a full chunk of
m = 64 with blocked sweeps on D2Q5 and D2Q9): sampled nodes against the
oracle on crops, as at the benchmark size.  The fields are smooth and separable, so that they
are cheap to build at this size and the crops see exactly the values the
GPU gets (float32 products and sums of float32 factors)."""
import time

import numpy as np
import pytest

from paper_1808_07554_amd import inputs
from tests.test_gpu_fullsize import K1_2D, K1_3D, _check_samples, _samples, reach

pytestmark = pytest.mark.gpu

def _axis(n, period, amp, phase, base=0.0):
    t = np.arange(n, dtype=np.float64)
    return (base + amp * np.sin(2 * np.pi * t / period + phase)).astype(np.float32)


def _fields(shape, lattice):
    """Smooth separable fields on [z][y][x]: K a product, phi a sum of float32
    factors per axis; P0 linear in x, S0 = 0."""
    params, _ = inputs.injection_problem((8, 8, 8) if lattice == "D3Q7" else (8, 8), 1.0, 4.0, 1, 2)
    dims = shape if lattice == "D3Q7" else shape[:2]
    params = dict(params, shape=tuple(shape) + (1,) * (3 - len(shape)))
    if lattice == "D2Q9":
        params = dict(params, lattice="D2Q9", beta=0.2)     # eq. 3-4: max(phi)/2 <= beta <= 2 min(phi)
    K0 = np.float32(params["mu_n"] / 6.0)
    kf = [np.exp(_axis(n, p, 0.4, f)).astype(np.float32) for n, p, f in zip(dims, (97.0, 61.0, 43.0), (0.0, 1.0, 2.0))]
    pf = [_axis(n, p, 0.02, f) for n, p, f in zip(dims, (53.0, 41.0, 37.0), (0.5, 1.5, 2.5))]
    pf[1] = pf[1] + np.float32(0.22)
    K, phi = kf[0] * K0, pf[0]
    for a in range(1, len(dims)):            # outer products / sums, slowest axis first
        K = np.multiply.outer(kf[a], K)
        phi = np.add.outer(pf[a], phi)
    x = np.arange(dims[0], dtype=np.float64)
    P0 = np.broadcast_to((1.0 - (x + 0.5) / dims[0]).astype(np.float32), K.shape).copy()
    S0 = np.zeros(K.shape, np.float32)
    fshape = (1,) + K.shape if lattice != "D3Q7" else K.shape
    fl = {k: v.reshape(fshape) for k, v in dict(K=K, phi=phi, P0=P0, S0=S0).items()}
    return params, fl


CASES = [
    ("D2Q5", (20480, 20960), 5, 3),     # 5 x 429 260 800 < 2^31, about 45 GB
    ("D2Q9", (15360, 15520), 9, 3),     # 9 x 238 387 200 < 2^31, about 40 GB
    ("D3Q7", (670, 670, 670), 7, 1),    # 7 x 300 763 000 < 2^31, about 40 GB
]


@pytest.mark.parametrize("lattice,shape,Q,n_interior", CASES)
def test_largest_problem_sampled_parity(lattice, shape, Q, n_interior):
    assert Q * int(np.prod(shape)) < 2 ** 31
    t0 = time.perf_counter()
    params, fl = _fields(shape, lattice)
    print(f"{lattice} {shape}: fields built in {time.perf_counter() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(29)
    k1 = K1_3D if lattice == "D3Q7" else K1_2D
    worst = _check_samples(params, fl, _samples(shape, rng, n_interior, reach(k1)), "fp32", k1)
    print(f"done in {time.perf_counter() - t0:.1f} s", flush=True)
    for k, v in worst.items():
        assert v <= 1e-5, (k, v)
