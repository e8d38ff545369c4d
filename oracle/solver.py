"""Plain CPU oracle of the double-distribution lattice Boltzmann model.

TEST INFRASTRUCTURE: part of the CPU oracle (see oracle/__init__.py).  Only
tests, the smoke check and the CPU-baseline leg of the benchmark use it.

Everything is whole-array NumPy in float64 (``dtype=np.float32`` gives a
diagnostic single-precision run of the same code; its reductions stay in
float64).  The algorithm follows the paper's order:

  coupled step n (physical time t_n = n dt)
    1. S^n from the g moments, eq. (3-9b); mobilities and D_p = K lambda_t,
       eq. (2-9), (2-16); tau_f(x) from eq. (3-11a); gamma(x) from eq. (3-8);
       tau_g from eq. (3-11b): a scalar for a constant D_s; with a capillary
       coefficient B > 0, D_s(x) = D_s + B K lambda_n f_w (eq. 2-16 with the
       linear capillary curve P_c = B (1 - S)) and tau_g(x) is a field.
    2. Pressure iteration in pseudo time, eq. (3-1) with eq. (3-3): moment
       P = sum_{i>=1} f_i / (1 - w_0) (eq. 3-9a), BGK collision (eq. 2-1b a),
       streaming, then the boundary rules of Section 4: anti-bounce-back for
       Dirichlet pressure, bounce-back for no flux.  Iterated until the
       stopping rule below holds ("iterated to reach a steady state",
       Section 3).  f carries over from one coupled step to the next.
    3. The local pressure gradient and velocity from the first moment of f,
       eq. (3-10), on the final pre-collision f.
    4. One step of the saturation lattice, eq. (3-2) with equilibrium
       eq. (3-4) (D2Q9) or eq. (3-4b) (D2Q5, D3Q7), using S^n, grad P^n and
       F_s(t_n); streaming; anti-bounce-back with g^eq(S_wb) for Dirichlet
       saturation, bounce-back for no flux.

Readings where the paper is silent (each is also listed in the design notes):
  * stopping rule: r_k = ||P^k - P^{k-m}||_2 / (m ||P^k||_2) with float64
    sums, evaluated when k is a positive multiple of m; stop at the first
    r_k <= tol, or after max_iters iterations.  ||P^k|| = 0 uses the
    absolute change.
  * f initialisation: f_i = w_i P0 - tau_f dt w_i c_i . grad P0 (i >= 1),
    the equilibrium plus the first-order Chapman-Enskog part of Appendix A;
    f_0 = (w_0 - 1) P0.
  * walls sit halfway between nodes (nodes at (j + 1/2) dx on walled axes,
    j dx on periodic axes); a boundary value given as a function is evaluated
    where and when the reflected population meets the wall: at the midpoint
    of the cut link and, for the saturation lattice, at t_n + dt/2 (the
    population leaves the node after the collision at t_n and is back at
    t_n + dt, so it is at the halfway wall half a step in between).  The
    pressure lattice iterates in pseudo time at the fixed physical time t_n,
    so its wall values are taken at t_n.
  * "outflow" for the saturation lattice is anti-bounce-back with
    S_wb = S^n at the boundary node (a zero-gradient outlet; the paper has
    only Dirichlet and no-flux walls).
  * the D2Q9 anti-bounce-back equilibrium uses phi at the boundary node.
  * collision: BGK as in the paper; optionally (D2Q9, pressure lattice) the
    multiple-relaxation-time form the paper says the model extends to, with
    the Lallemand-Luo moment basis (lattice.d2q9_moment_basis), the fluxes
    relaxed at 1/tau_f and the other rates given (rho, e, epsilon share one).
  * a face may mix rules link by link (wells on a no-flux wall, the
    five-spot problem of Section 4.3): a predicate of the cut link's
    midpoint picks one of two rules for that link.
  * gradients of the initial fields, when not given, are second-order central
    differences (one-sided second order next to walls).
"""
import math

import numpy as np

from . import lattice as _lat

FACES = ("-x", "+x", "-y", "+y", "-z", "+z")

OK, NOT_CONVERGED, UNSTABLE = 0, 1, -4


class QuadraticKr:
    """k_rw = S^2, k_rn = (1 - S)^2 (Section 4.3) with lambda = k_r / mu (eq. 2-9).

    Returns D_p = K lambda_t (eq. 2-16) and lambda_w K (the coefficient of
    eq. 2-18 and eq. 3-8).
    """

    def __init__(self, mu_w, mu_n):
        self.mu_w, self.mu_n = float(mu_w), float(mu_n)

    def __call__(self, S, K):
        lam_w = S * S / self.mu_w
        lam_n = (1.0 - S) * (1.0 - S) / self.mu_n
        return K * (lam_w + lam_n), K * lam_w


class GivenCoefficients:
    """D_p(S) and lambda_w K(S) given directly (Examples 1 and 2, Section 4)."""

    def __init__(self, Dp, lamwK):
        self.Dp, self.lamwK = Dp, lamwK

    def __call__(self, S, K):
        return self.Dp(S), self.lamwK(S)


class Solver:
    """One lattice-Boltzmann realisation on a box of nx x ny (x nz) nodes.

    bc_f[face] is ("periodic",), ("abb", P_b) or ("bb",);
    bc_g[face] is ("periodic",), ("abb", S_b), ("bb",) or ("outflow",).
    A boundary value may be a number or a function of (x, y, z, t).
    Either face rule may also be ("links", pick, rule_a, rule_b): each cut
    link takes rule_a where pick(x, y, z, t) is true at its midpoint and
    rule_b elsewhere (neither of them periodic).
    """

    def __init__(self, lattice, shape, *, beta, Ds, coef, bc_f, bc_g,
                 dx=1.0, dt=1.0, m=1, dtype=np.float64, cap_B=0.0, collision=None):
        self.lat = _lat.get(lattice) if isinstance(lattice, str) else lattice
        shape = tuple(int(s) for s in shape)
        if len(shape) == 2:
            shape = shape + (1,)
        self.nx, self.ny, self.nz = shape
        if self.lat.dim == 2 and self.nz != 1:
            raise ValueError("2-D lattice needs nz = 1")
        self.fshape = (self.nz, self.ny, self.nx)
        self.dtype = np.dtype(dtype)
        self.dx, self.dt = float(dx), float(dt)
        self.c = self.dx / self.dt
        self.cs2 = self.lat.cs2_c2 * self.c * self.c
        self.beta, self.Ds = float(beta), float(Ds)
        self.cap_B = float(cap_B)
        # pressure-lattice collision: BGK (None), or ("mrt", s0, sq, sp) on D2Q9
        self.mrt = None
        if collision is not None:
            if collision[0] != "mrt" or len(collision) != 4 or self.lat.name != "D2Q9":
                raise ValueError("collision: None or ('mrt', s0, sq, sp) on D2Q9")
            rates = [float(v) for v in collision[1:]]
            if not all(0.0 < v < 2.0 for v in rates):
                raise ValueError("MRT rates must lie in (0, 2)")
            M = _lat.d2q9_moment_basis()
            self.mrt = (M, np.linalg.inv(M), rates)
        if self.cap_B < 0:
            raise ValueError("capillary coefficient must be non-negative")
        self.coef = coef
        self.m = int(m)
        self.bc_f = [tuple(b) for b in bc_f]
        self.bc_g = [tuple(b) for b in bc_g]
        if len(self.bc_f) != 2 * self.lat.dim or len(self.bc_g) != 2 * self.lat.dim:
            raise ValueError("one boundary condition per face")
        for a in range(self.lat.dim):
            per = [b[0] == "periodic" for b in
                   (self.bc_f[2 * a], self.bc_f[2 * a + 1], self.bc_g[2 * a], self.bc_g[2 * a + 1])]
            if any(per) and not all(per):
                raise ValueError("periodicity must hold on both faces of an axis for f and g")
        # tau_g from eq. (3-11b); validity: tau > 1/2 and non-negative g^eq
        self.tau_g = self._tau_g(self.Ds)
        if not self.tau_g > 0.5:
            raise ValueError("tau_g must exceed 1/2")
        self.t = 0.0
        self.n = 0
        self.flux_ledger = 0.0
        self.g_bc_time = 0.5
        self._coords()

    # ------------------------------------------------------------------ setup
    def _coords(self):
        ax = []
        for a, n in enumerate((self.nx, self.ny, self.nz)):
            periodic = a >= self.lat.dim or self.bc_f[2 * a][0] == "periodic"
            off = 0.0 if periodic else 0.5
            ax.append((np.arange(n) + off) * self.dx)
        z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        self.X, self.Y, self.Z = x, y, z

    def _field(self, v, default=0.0):
        if v is None:
            v = default
        a = np.asarray(v, dtype=np.float64)
        if a.ndim == 0:
            a = np.full(self.fshape, float(a))
        return a.reshape(self.fshape).astype(self.dtype)

    def set_fields(self, K, phi, Fp=None, Fs=None):
        """Absolute permeability K(x), porosity phi(x) and the sources F_p, F_s (eq. 2-17)."""
        self.K = self._field(K)
        self.phi = self._field(phi)
        if np.any(self.K <= 0) or np.any(self.phi <= 0):
            raise ValueError("K and phi must be positive")
        if self.lat.odd:
            bmax = float(self.phi.min()) / (1.0 - self.lat.w[0])    # eq. (3-4b) bound
            if not (0.0 <= self.beta <= bmax + 1e-15):
                raise ValueError("beta outside [0, phi/(1-w0)]")
        else:
            if not (np.all(self.phi / 2 <= self.beta) and np.all(self.beta <= 2 * self.phi)):
                raise ValueError("beta outside [phi/2, 2 phi]")      # eq. (3-4) bound
        self.set_sources(Fp, Fs)

    def set_sources(self, Fp=None, Fs=None):
        self.Fp = self._field(Fp)
        self.Fs = self._field(Fs)

    # ------------------------------------------------------------- equilibria
    def _ev(self, i):
        """c_i as a 3-vector of floats."""
        return self.lat.e[i].astype(np.float64) * self.c

    def feq(self, P):
        """eq. (3-3)."""
        lat = self.lat
        out = np.empty((lat.Q,) + self.fshape, dtype=self.dtype)
        out[0] = (lat.w[0] - 1.0) * P
        for i in range(1, lat.Q):
            out[i] = lat.w[i] * P
        return out

    def geq_i(self, i, S, phi):
        """g_i^eq: eq. (3-4) for D2Q9, eq. (3-4b) for the DnQ(2n+1) lattices."""
        lat = self.lat
        if lat.odd:
            if i == 0:
                return ((lat.w[0] - 1.0) * self.beta + phi) * S
            return lat.w[i] * self.beta * S
        ci = self._ev(i)
        # C:(c_i c_i - cs^2 I) with C = (beta - phi) I
        contr = (self.beta - phi) * (ci @ ci - lat.dim * self.cs2)
        return lat.w[i] * S * (phi + contr / (2.0 * self.cs2))

    def geq(self, S):
        return np.stack([self.geq_i(i, S, self.phi) for i in range(self.lat.Q)]).astype(self.dtype)

    # --------------------------------------------------------------- moments
    def pressure(self):
        """eq. (3-9a) on the current pre-collision f."""
        return self.f[1:].sum(axis=0) / (1.0 - self.lat.w[0])

    def saturation(self):
        """eq. (3-9b) on the current pre-collision g with the current F_s."""
        return (self.g.sum(axis=0) + 0.5 * self.dt * self.Fs) / self.phi

    def grad_p(self):
        """Local pressure gradient, eq. (3-10a): -sum_i c_i f_i / (tau_f dt c_s^2)."""
        m1 = np.zeros((3,) + self.fshape, dtype=self.dtype)
        for i in range(1, self.lat.Q):
            ci = self._ev(i)
            for a in range(3):
                if ci[a] != 0.0:
                    m1[a] += ci[a] * self.f[i]
        return -m1 / (self.tau_f * self.dt * self.cs2)

    def velocity(self):
        """eq. (3-10b): u = -K lambda_t grad P with K lambda_t = D_p at S^n."""
        return -self.Dp * self.grad_p()

    def phase_velocities(self):
        """Phase velocities of eq. (2-12), (2-13) at S^n:
            u_w = f_w (u + K lambda_n grad P_c),  u_n = f_n (u - K lambda_w grad P_c),
        with f_w = lambda_w / lambda_t = (lambda_w K) / D_p (eq. 2-10).  The
        saturation diffusivity of eq. (2-16), D_s = -K lambda_n f_w P_c'(S),
        is the constant D_s of the model, so K lambda_n grad P_c =
        K lambda_n P_c' grad S = -(D_s / f_w) grad S and
            u_w = f_w u - D_s grad S,  u_n = f_n u + D_s grad S.
        grad S by second-order central differences (one-sided at walls)."""
        u = self.velocity()
        fw = self.lamwK / self.Dp
        gS = self._cdiff(self.S.astype(np.float64))
        uw = fw * u - self.Ds * gS
        un = (1.0 - fw) * u + self.Ds * gS
        return uw, un

    def mass(self):
        """M = sum_x phi S (float64), and the accumulated boundary-link flux of g."""
        return float(np.sum((self.phi * self.saturation()).astype(np.float64))), self.flux_ledger

    # ---------------------------------------------------------- coefficients
    def _tau_g(self, Ds):
        """eq. (3-11b)."""
        return 0.5 + Ds / (self.beta * self.cs2 * self.dt)

    def saturation_diffusivity(self, S, Dp, lamwK):
        """D_s of eq. (2-16), D_s = -K lambda_n f_w dP_c/dS, for the capillary
        curve P_c = B (1 - S) on top of the constant D_s of the model:
        D_s + B K lambda_n f_w with K lambda_n = D_p - lambda_w K and
        f_w = lambda_w K / D_p (eq. 2-10)."""
        if self.cap_B == 0.0:
            return self.Ds
        return self.Ds + self.cap_B * (Dp - lamwK) * (lamwK / Dp)

    def update_coefficients(self):
        """S^n, D_p, tau_f(x), gamma(x) and tau_g (field with a capillary
        term) for the current coupled step."""
        self.S = self.saturation()
        self.Dp, self.lamwK = self.coef(self.S, self.K)
        if self.cap_B != 0.0:
            self.tau_g = self._tau_g(self.saturation_diffusivity(self.S, *self.coef(self.S, self.K)))
        self.Dp = np.asarray(self.Dp, dtype=self.dtype) * np.ones(self.fshape, self.dtype)
        self.lamwK = np.asarray(self.lamwK, dtype=self.dtype) * np.ones(self.fshape, self.dtype)
        self.tau_f = 0.5 + self.Dp / (self.cs2 * self.dt)          # eq. (3-11a)
        self.gamma = -self.lamwK / (self.cs2 * self.dt)            # eq. (3-8)
        if not np.all(self.tau_f > 0.5):
            raise FloatingPointError("tau_f <= 1/2")

    # ------------------------------------------------------------ streaming
    def _bvalue(self, v, i, sl, t):
        """Boundary value at the midpoints of the links cut at cells sl."""
        if callable(v):
            h = 0.5 * self.lat.e[i].astype(np.float64) * self.dx
            return v(self.X[sl] - h[0], self.Y[sl] - h[1], self.Z[sl] - h[2], t)
        return float(v)

    def _stream(self, post, bcs, wall_value, t):
        """Streaming: new_i(x) = post_i(x - c_i dt), with the wall rules where x - c_i
        lies outside the box.  wall_value(i, b, sl, t) gives the ABB term of face rule b.

        Returns the new populations and the net flux the wall rules let in:
        sum over cut links of new_i(x_f) - post_{opp i}(x_f).
        """
        lat = self.lat
        new = np.empty_like(post)
        flux = 0.0
        axes = (2, 1, 0)        # x, y, z axes of a [z][y][x] field
        for i in range(lat.Q):
            ei = lat.e[i]
            v = post[i]
            for a in range(3):
                if ei[a] != 0:
                    v = np.roll(v, int(ei[a]), axis=axes[a])
            v = v.copy()
            mask = np.zeros(self.fshape, dtype=bool)
            for a in range(lat.dim):
                if ei[a] == 0:
                    continue
                face = 2 * a + (0 if ei[a] > 0 else 1)
                b = bcs[face]
                if b[0] == "periodic":
                    continue
                sl = [slice(None)] * 3
                sl[axes[a]] = 0 if ei[a] > 0 else -1
                sl = tuple(sl)
                v[sl] = self._wall_rule(b, i, sl, post[lat.opp[i]][sl], wall_value, t)
                mask[sl] = True
            if mask.any():
                flux += float(np.sum(v[mask].astype(np.float64) - post[lat.opp[i]][mask].astype(np.float64)))
            new[i] = v
        return new, flux

    def _wall_rule(self, b, i, sl, src, wall_value, t):
        """Population i arriving through a wall at cells sl (Section 4):
        bounce-back gives the reflected post-collision population src,
        anti-bounce-back -src plus the equilibrium term of the face value."""
        if b[0] == "bb":
            return src
        if b[0] in ("abb", "outflow"):
            return -src + wall_value(i, b, sl, t)
        if b[0] == "links":
            pick = np.broadcast_to(self._bvalue(b[1], i, sl, t), src.shape)
            return np.where(pick, self._wall_rule(b[2], i, sl, src, wall_value, t),
                            self._wall_rule(b[3], i, sl, src, wall_value, t))
        raise ValueError(b)

    # ------------------------------------------------------- pressure lattice
    def _f_wall(self, i, b, sl, t):
        j = self.lat.opp[i]
        return 2.0 * self.lat.w[j] * self._bvalue(b[1], i, sl, t)

    def _mrt_relax(self, neq):
        """M^-1 S M (f - f^eq): the multiple-relaxation-time collision the paper
        says the model extends to (Section 3).  Rates: s0 for rho, e and epsilon
        (equal, so the rest population, which no output uses, stays decoupled
        from the moving ones), 1/tau_f for the fluxes j_x, j_y (they carry the
        diffusivity, eq. 3-11a), sq for q_x, q_y and sp for p_xx, p_xy."""
        M, Minv, (s0, sq, sp) = self.mrt
        m = np.einsum("ki,i...->k...", M, neq)
        sj = 1.0 / self.tau_f
        rates = [s0, s0, s0, sj, sq, sj, sq, sp, sp]
        sm = np.stack([r * m[k] for k, r in enumerate(rates)])
        return np.einsum("ik,k...->i...", Minv, sm)

    def f_iteration(self):
        """One iteration of eq. (3-1): collide (eq. 2-1b a), stream, wall rules."""
        lat = self.lat
        P = self.pressure()
        if self.mrt is None:
            post = self.f - (self.f - self.feq(P)) / self.tau_f
        else:
            post = self.f - self._mrt_relax(self.f - self.feq(P))
        for i in range(1, lat.Q):
            post[i] = post[i] + self.dt * lat.wbar[i] * self.Fp
        self.f, _ = self._stream(post, self.bc_f, self._f_wall, self.t)

    def pressure_solve(self, tol, max_iters):
        """Iterate eq. (3-1) at the current S^n.  Returns (iterations, r, status)."""
        m = self.m
        P_snap = self.pressure().astype(np.float64)
        r = math.inf
        k = 0
        while k < max_iters:
            self.f_iteration()
            k += 1
            if k % m == 0:
                Pk = self.pressure().astype(np.float64)
                num = math.sqrt(float(np.sum((Pk - P_snap) ** 2)))
                den = math.sqrt(float(np.sum(Pk ** 2)))
                r = num / (m * den) if den > 0 else num / m
                P_snap = Pk
                if not math.isfinite(r):
                    return k, r, UNSTABLE
                if r <= tol:
                    return k, r, OK
        return k, r, NOT_CONVERGED

    # ----------------------------------------------------- saturation lattice
    def _g_wall(self, i, b, sl, t):
        j = self.lat.opp[i]
        if b[0] == "outflow":
            Sb = self.S[sl]
        else:
            Sb = self._bvalue(b[1], i, sl, t)
        return 2.0 * self.geq_i(j, Sb, self.phi[sl])

    def saturation_step(self):
        """One step of eq. (3-2) with S^n, the local grad P^n and F_s(t_n)."""
        lat = self.lat
        S = self.S
        gp = self.grad_p()
        tg = self.tau_g
        geq = self.geq(S)
        post = self.g - (self.g - geq) / tg
        for i in range(lat.Q):
            ci = self._ev(i)
            cdg = ci[0] * gp[0] + ci[1] * gp[1] + ci[2] * gp[2]
            post[i] = (post[i] + self.dt * lat.w[i] * (1.0 - 1.0 / (2.0 * tg)) * self.Fs
                       + self.gamma * self.dt * lat.w[i] * cdg / tg)
        self.g, flux = self._stream(post, self.bc_g, self._g_wall, self.t + self.g_bc_time * self.dt)
        self.flux_ledger += flux
        self.n += 1
        self.t = self.n * self.dt

    def step(self, tol, max_iters, sources=None):
        """One coupled step: coefficients at S^n, pressure solve, saturation step.

        sources(t) -> (F_p, F_s), if given, is applied before the step.
        Returns the pressure iteration count.
        """
        if sources is not None:
            self.set_sources(*sources(self.t))
        self.update_coefficients()
        k, r, st = self.pressure_solve(tol, max_iters)
        if st == UNSTABLE:
            raise FloatingPointError("non-finite residual")
        self.last = (k, r, st)
        self.saturation_step()
        return k

    # --------------------------------------------------------- initialisation
    def _cdiff(self, u):
        """Second-order central differences (one-sided second order at walls;
        the three-point one-sided formula needs three nodes along a walled
        axis, and a shorter one is refused)."""
        g = np.zeros((3,) + self.fshape)
        axes = (2, 1, 0)
        for a in range(self.lat.dim):
            ax = axes[a]
            if self.bc_f[2 * a][0] != "periodic" and u.shape[ax] < 3:
                raise ValueError("a walled axis needs at least three nodes (one-sided differences)")
            if self.bc_f[2 * a][0] == "periodic":
                g[a] = (np.roll(u, -1, ax) - np.roll(u, 1, ax)) / (2 * self.dx)
            else:
                d = (np.roll(u, -1, ax) - np.roll(u, 1, ax)) / (2 * self.dx)
                n = u.shape[ax]
                take = lambda j: np.take(u, [j], axis=ax)
                lo = (-3 * take(0) + 4 * take(1) - take(2)) / (2 * self.dx)
                hi = (3 * take(n - 1) - 4 * take(n - 2) + take(n - 3)) / (2 * self.dx)
                sl = [slice(None)] * 3
                sl[ax] = slice(0, 1)
                d[tuple(sl)] = lo
                sl[ax] = slice(n - 1, n)
                d[tuple(sl)] = hi
                g[a] = d
        return g

    def set_state(self, P0, S0, dP0=None, dS0=None, neq=True):
        """Initial populations (initialisation paragraph of Section 4).

        g_i = g_i^eq(S0) + eps g_i^(1) with eps g_i^(1) from the Chapman-Enskog
        expansion (eq. gneq); f_i = f_i^eq(P0) plus the first-order part
        -tau_f dt w_i c_i . grad P0.  dP0, dS0: (3, nz, ny, nx) gradients, or None
        for central differences.  neq=False gives pure equilibria.
        """
        lat = self.lat
        P0 = self._field(P0)
        S0 = self._field(S0)
        dP0 = self._cdiff(P0.astype(np.float64)) if dP0 is None else np.asarray(dP0, np.float64).reshape((3,) + self.fshape)
        dS0 = self._cdiff(S0.astype(np.float64)) if dS0 is None else np.asarray(dS0, np.float64).reshape((3,) + self.fshape)
        dP0 = dP0.astype(self.dtype)
        dS0 = dS0.astype(self.dtype)
        Dp, lamwK = self.coef(S0, self.K)
        tau_f = 0.5 + Dp / (self.cs2 * self.dt)
        gamma = -lamwK / (self.cs2 * self.dt)
        tg = self._tau_g(self.saturation_diffusivity(S0, Dp, lamwK))
        f = self.feq(P0)
        g = self.geq(S0)
        if neq:
            for i in range(1, lat.Q):
                ci = self._ev(i)
                cdp = ci[0] * dP0[0] + ci[1] * dP0[1] + ci[2] * dP0[2]
                f[i] = f[i] - tau_f * self.dt * lat.w[i] * cdp
            for i in range(lat.Q):
                ci = self._ev(i)
                cdp = ci[0] * dP0[0] + ci[1] * dP0[1] + ci[2] * dP0[2]
                cds = ci[0] * dS0[0] + ci[1] * dS0[1] + ci[2] * dS0[2]
                Gam = self.geq_i(i, 1.0, self.phi)      # Gamma_i = g_i^eq / S
                g1 = ((Gam / self.phi - lat.w[i] * (1.0 - 1.0 / (2.0 * tg))) * self.Fs
                      + Gam * cds - gamma * lat.w[i] * cdp / tg)
                g[i] = g[i] - tg * self.dt * g1
        self.f = f.astype(self.dtype)
        self.g = g.astype(self.dtype)
        self.t = 0.0
        self.n = 0
        self.flux_ledger = 0.0
