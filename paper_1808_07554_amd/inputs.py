"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the CPU oracle.

This module holds no lattice Boltzmann arithmetic: it only draws random
fields and evaluates closed-form manufactured solutions of the macroscopic
two-phase Darcy model (the global-pressure Poisson equation eq. (2-15) and
the saturation equation eq. (2-18)) together with the source terms that make
them exact.  Both sides of every parity check receive exactly the arrays
produced here (float64, then rounded once to float32 where the GPU path
stores float32).

Workloads (lattice units, dx = dt = 1 unless stated):
  * ``manufactured_periodic``: a periodic square, homogeneous K = 1,
    phi = 0.2, mu_w = 1, mu_n = 5, quadratic relative permeabilities,
    beta = 0.2, D_s = 1/30 (tau_g = 1); exact P_e = 0.1 sin(kx) sin(ky),
    S_e = 0.5 + 0.1 cos(kx) cos(ky) cos(w t) with k = 2 pi / N, w = 2 pi / 1000.
  * ``injection``: log-normal permeability from a seeded Gaussian random
    field, porosity uniform in [0.15, 0.3], mu_w = 1, mu_n = 5, quadratic
    relative permeabilities, pressure 1 and saturation 1 imposed on the x = 0
    face, pressure 0 and a zero-gradient saturation outlet on the x = L face,
    no flux on the other faces, S0 = 0, P0 the linear ramp.
  * ``five_spot``: the quarter five-spot of Section 4.3 (Table 1 values) on
    the unit square, D2Q9; injection and production wells as short
    Dirichlet segments of the walls at opposite corners (see five_spot).
"""
import math

import numpy as np

FACES = ("-x", "+x", "-y", "+y", "-z", "+z")


def gaussian_random_field(shape, ell, seed):
    """Periodic Gaussian random field with covariance exp(-r^2 / ell^2) (ell in cells).

    Spectral synthesis: white noise xi ~ N(0, 1) from numpy's PCG64 generator,
    filtered by sqrt(S(k)) with S(k) ~ exp(-|k|^2 ell^2 / 4), then shifted and
    scaled to sample mean 0 and variance 1.  shape is (nz, ny, nx) or (ny, nx).
    """
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(shape)
    F = np.fft.rfftn(xi)
    k2 = np.zeros(F.shape)
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = 2 * np.pi * np.fft.rfftfreq(n)
        else:
            k = 2 * np.pi * np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = len(k)
        k2 = k2 + (k.reshape(sh)) ** 2
    F *= np.exp(-k2 * ell * ell / 8.0)          # sqrt of the spectrum
    z = np.fft.irfftn(F, s=shape, axes=tuple(range(len(shape))))
    z -= z.mean()
    z /= z.std()
    return z


def uniform_field(shape, lo, hi, seed):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


# ----------------------------------------------------------------------------
# Manufactured periodic problem
# ----------------------------------------------------------------------------
class ManufacturedPeriodic:
    """Exact smooth solution of eq. (2-15) and eq. (2-18) on a periodic N x N box.

    Nodes sit at integer positions (x, y) = (i, j).  All quantities float64.
    """

    def __init__(self, N=64, amp_p=0.1, amp_s=0.1, period=1000.0, K=1.0, phi=0.2,
                 mu_w=1.0, mu_n=5.0, beta=0.2, Ds=1.0 / 30.0):
        self.N = N
        self.k = 2 * np.pi / N
        self.w = 2 * np.pi / period
        self.ap, self.as_ = amp_p, amp_s
        self.K, self.phi, self.mu_w, self.mu_n = K, phi, mu_w, mu_n
        self.beta, self.Ds = beta, Ds
        j = np.arange(N, dtype=np.float64)
        self.Y, self.X = np.meshgrid(j, j, indexing="ij")      # [y][x]

    def _trig(self):
        k = self.k
        return (np.sin(k * self.X), np.cos(k * self.X), np.sin(k * self.Y), np.cos(k * self.Y))

    def P(self):
        sx, cx, sy, cy = self._trig()
        return self.ap * sx * sy

    def gradP(self):
        sx, cx, sy, cy = self._trig()
        return np.stack([self.ap * self.k * cx * sy, self.ap * self.k * sx * cy, 0 * sx])

    def S(self, t):
        sx, cx, sy, cy = self._trig()
        return 0.5 + self.as_ * cx * cy * math.cos(self.w * t)

    def gradS(self, t):
        sx, cx, sy, cy = self._trig()
        a = -self.as_ * self.k * math.cos(self.w * t)
        return np.stack([a * sx * cy, a * cx * sy, 0 * sx])

    def velocity(self, t):
        """u = -K lambda_t(S_e) grad P_e (eq. 2-7)."""
        S = self.S(t)
        lam_t = S * S / self.mu_w + (1 - S) ** 2 / self.mu_n
        return -self.K * lam_t * self.gradP()

    def sources(self, t):
        """(F_p, F_s) making (P_e, S_e) exact for eq. (2-15) and eq. (2-18)."""
        S = self.S(t)
        P = self.P()
        lap_p = -2 * self.k ** 2 * P
        lap_s = -2 * self.k ** 2 * (S - 0.5)
        gs, gp = self.gradS(t), self.gradP()
        gsgp = gs[0] * gp[0] + gs[1] * gp[1]
        sx, cx, sy, cy = self._trig()
        dSdt = -self.as_ * self.w * cx * cy * math.sin(self.w * t)
        lam_w = S * S / self.mu_w
        lam_t = lam_w + (1 - S) ** 2 / self.mu_n
        dlam_w = 2 * S / self.mu_w
        dlam_t = dlam_w - 2 * (1 - S) / self.mu_n
        Fp = -self.K * (lam_t * lap_p + dlam_t * gsgp)
        Fs = self.phi * dSdt - self.Ds * lap_s - self.K * (lam_w * lap_p + dlam_w * gsgp)
        return Fp, Fs


class ManufacturedPeriodic3D:
    """The manufactured problem of ManufacturedPeriodic on a periodic N^3 box:
    P_e = a sin(kx) sin(ky) sin(kz), S_e = 0.5 + b cos(kx) cos(ky) cos(kz) cos(w t),
    with the sources that make them exact for eq. (2-15) and eq. (2-18).
    Nodes at integer positions; fields are [z][y][x], float64."""

    def __init__(self, N=16, amp_p=0.1, amp_s=0.1, period=1000.0, K=1.0, phi=0.2,
                 mu_w=1.0, mu_n=5.0, beta=0.15, Ds=0.01875):
        self.N = N
        self.k = 2 * np.pi / N
        self.w = 2 * np.pi / period
        self.ap, self.as_ = amp_p, amp_s
        self.K, self.phi, self.mu_w, self.mu_n = K, phi, mu_w, mu_n
        self.beta, self.Ds = beta, Ds
        j = np.arange(N, dtype=np.float64)
        self.Z, self.Y, self.X = np.meshgrid(j, j, j, indexing="ij")

    def _trig(self):
        k = self.k
        return [(np.sin(k * a), np.cos(k * a)) for a in (self.X, self.Y, self.Z)]

    def P(self):
        (sx, _), (sy, _), (sz, _) = self._trig()
        return self.ap * sx * sy * sz

    def gradP(self):
        (sx, cx), (sy, cy), (sz, cz) = self._trig()
        a = self.ap * self.k
        return np.stack([a * cx * sy * sz, a * sx * cy * sz, a * sx * sy * cz])

    def S(self, t):
        (_, cx), (_, cy), (_, cz) = self._trig()
        return 0.5 + self.as_ * cx * cy * cz * math.cos(self.w * t)

    def gradS(self, t):
        (sx, cx), (sy, cy), (sz, cz) = self._trig()
        a = -self.as_ * self.k * math.cos(self.w * t)
        return np.stack([a * sx * cy * cz, a * cx * sy * cz, a * cx * cy * sz])

    def velocity(self, t):
        S = self.S(t)
        lam_t = S * S / self.mu_w + (1 - S) ** 2 / self.mu_n
        return -self.K * lam_t * self.gradP()

    def sources(self, t):
        S = self.S(t)
        lap_p = -3 * self.k ** 2 * self.P()
        lap_s = -3 * self.k ** 2 * (S - 0.5)
        gsgp = np.sum(self.gradS(t) * self.gradP(), axis=0)
        (_, cx), (_, cy), (_, cz) = self._trig()
        dSdt = -self.as_ * self.w * cx * cy * cz * math.sin(self.w * t)
        lam_w = S * S / self.mu_w
        lam_t = lam_w + (1 - S) ** 2 / self.mu_n
        dlam_w = 2 * S / self.mu_w
        dlam_t = dlam_w - 2 * (1 - S) / self.mu_n
        Fp = -self.K * (lam_t * lap_p + dlam_t * gsgp)
        Fs = self.phi * dSdt - self.Ds * lap_s - self.K * (lam_w * lap_p + dlam_w * gsgp)
        return Fp, Fs


def manufactured_problem(N=64):
    """Parameters of the manufactured periodic workload as a plain dict."""
    m = ManufacturedPeriodic(N)
    return dict(lattice="D2Q5", shape=(N, N, 1), dx=1.0, dt=1.0, beta=m.beta, Ds=m.Ds,
                mu_w=m.mu_w, mu_n=m.mu_n,
                bc_f=[("periodic",)] * 4, bc_g=[("periodic",)] * 4), m


# ----------------------------------------------------------------------------
# Heterogeneous injection problem (2-D and 3-D)
# ----------------------------------------------------------------------------
def injection_problem(shape, sigma, ell, seed_k, seed_phi, K0=None, beta=0.15, Ds=None,
                      mu_w=1.0, mu_n=5.0):
    """Inputs of the heterogeneous injection workload.

    shape = (nx, ny) or (nx, ny, nz).  K0 and D_s default to the values that
    make both relaxation times 1 at the reference cell (c_s^2 = 1/3 in 2-D,
    1/4 in 3-D): K0 = c_s^2 mu_n / 2, D_s = beta c_s^2 / 2.
    Returns (params dict, fields dict) with float64 arrays laid out [z][y][x].
    """
    shape = tuple(shape)
    three_d = len(shape) == 3 and shape[2] > 1
    nx, ny = shape[0], shape[1]
    nz = shape[2] if three_d else 1
    cs2 = 0.25 if three_d else 1.0 / 3.0
    if K0 is None:
        K0 = cs2 * mu_n / 2
    if Ds is None:
        Ds = beta * cs2 / 2
    fshape = (nz, ny, nx) if three_d else (ny, nx)
    lnK = sigma * gaussian_random_field(fshape, ell, seed_k)
    K = K0 * np.exp(lnK)
    phi = uniform_field(fshape, 0.15, 0.3, seed_phi)
    x = (np.arange(nx) + 0.5) / nx
    P0 = np.broadcast_to(1.0 - x, fshape).copy()
    S0 = np.zeros(fshape)
    nfaces = 6 if three_d else 4
    bc_f = [("abb", 1.0), ("abb", 0.0)] + [("bb",)] * (nfaces - 2)
    bc_g = [("abb", 1.0), ("outflow",)] + [("bb",)] * (nfaces - 2)
    params = dict(lattice="D3Q7" if three_d else "D2Q5", shape=(nx, ny, nz), dx=1.0, dt=1.0,
                  beta=beta, Ds=Ds, mu_w=mu_w, mu_n=mu_n, bc_f=bc_f, bc_g=bc_g)
    fields = dict(K=K.reshape(nz, ny, nx), phi=phi.reshape(nz, ny, nx),
                  P0=P0.reshape(nz, ny, nx), S0=S0.reshape(nz, ny, nx), lnK=lnK.reshape(nz, ny, nx))
    return params, fields


def injection_2d(n=4096, sigma=1.0, ell=16.0, seed_k=2, seed_phi=3):
    return injection_problem((n, n), sigma, ell, seed_k, seed_phi)


def injection_3d(n=512, sigma=1.5, ell=8.0, seed_k=4, seed_phi=5):
    return injection_problem((n, n, n), sigma, ell, seed_k, seed_phi)


def f32(a):
    """Round once to float32 (the storage type of the GPU fields)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def ensemble(n_members=256, seed0=5000, sizes=(128, 256, 512, 1024), sigma_range=(0.5, 2.0), ell=16.0):
    """Ensemble of independent 2-D injection realisations of uneven size.

    Member j: side n_j drawn uniformly from `sizes`, sigma_lnK uniform in
    sigma_range (both from a PCG64 generator seeded seed0 + j), its own
    log-normal permeability field (seed 2 * (seed0 + j)) and porosity field
    (seed 2 * (seed0 + j) + 1).  Returns a list of (params, fields).
    """
    out = []
    for j in range(n_members):
        rng = np.random.default_rng(seed0 + j)
        n = int(rng.choice(sizes))
        sigma = float(rng.uniform(*sigma_range))
        out.append(injection_problem((n, n), sigma, ell, 2 * (seed0 + j), 2 * (seed0 + j) + 1))
    return out


# ----------------------------------------------------------------------------
# Five-spot problem (Section 4.3)
# ----------------------------------------------------------------------------
FIVE_SPOT_WELL = 0.12


def five_spot(N=96, well=FIVE_SPOT_WELL, P_inj=1.0, P_prod=0.0, beta=1.0, tau_g=1.0):
    """Inputs of the quarter five-spot problem of Section 4.3.

    Table 1: phi = 1, mu_w = mu_n = 1e-3, K = 1e-5, D_s = 1e-2, quadratic
    relative permeabilities, on [0, 1]^2.  The figure with the well layout is
    not available, so the layout here is the usual quarter pattern: the
    injector at corner (0, 0), the producer at (1, 1), each a Dirichlet
    segment of the two walls meeting at its corner: every link whose
    midpoint lies within `well` of the corner along the wall (0.12, so
    that no midpoint falls on a segment end at N = 32, 64, 96 and each
    segment is 1/8 long there).  Injector: P = P_inj and S_w = 1; producer:
    P = P_prod and a zero-gradient saturation outlet; no flux elsewhere.
    S0 = 0, P0 = P_inj + (P_prod - P_inj)(x + y)/2.  Lattice: N x N nodes,
    dx = 1/N, and c = 3 D_s / (beta (tau_g - 1/2) dx) so that the saturation
    relaxation time is tau_g at every N (diffusive scaling, dt ~ dx^2).
    Returns (params dict, fields dict) with float64 arrays laid out [z][y][x].
    """
    K0, phi0, mu, Ds = 1e-5, 1.0, 1e-3, 1e-2
    dx = 1.0 / N
    c = 3.0 * Ds / (beta * (tau_g - 0.5) * dx)
    dt = dx / c

    def inj(x, y, z, t):
        return (x < well) & (y < well)

    def prod(x, y, z, t):
        return (x > 1.0 - well) & (y > 1.0 - well)

    # faces -x, +x, -y, +y
    bc_f = [("links", inj, ("abb", P_inj), ("bb",)), ("links", prod, ("abb", P_prod), ("bb",))] * 2
    bc_g = [("links", inj, ("abb", 1.0), ("bb",)), ("links", prod, ("outflow",), ("bb",)),
            ("links", inj, ("abb", 1.0), ("bb",)), ("links", prod, ("outflow",), ("bb",))]
    x = (np.arange(N) + 0.5) * dx
    X, Y = np.meshgrid(x, x)
    params = dict(lattice="D2Q9", shape=(N, N, 1), dx=dx, dt=dt, beta=beta, Ds=Ds, mu_w=mu, mu_n=mu,
                  bc_f=bc_f, bc_g=bc_g)
    fields = dict(K=np.full((1, N, N), K0), phi=np.full((1, N, N), phi0),
                  P0=(P_inj + (P_prod - P_inj) * (X + Y) / 2).reshape(1, N, N), S0=np.zeros((1, N, N)))
    return params, fields
