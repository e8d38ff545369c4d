"""The paper's Examples 1 and 2 (Section 4.1, 4.2) as oracle runs.

Both use the D2Q9 lattice of Section 3, anti-bounce-back Dirichlet data from
the exact solutions on all four walls, initial data from the exact
solutions (with exact gradients for the non-equilibrium parts), and the
global relative L1 error E of Section 4.  With out={} the pressure iteration
counts of every coupled step (and of the final solve) and the solver are
returned in it, so the GPU can replay the run.
"""
import numpy as np

import oracle


def rel_l1(exact, num):
    return float(np.abs(exact - num).sum() / np.abs(exact).sum())


def example1(N, c=1.0, T=1.0, tol=1e-12, max_iters=500000, out=None):
    """Example 1: decoupled problem on [0,2]^2, phi = 1, D_p = D_s = 0.001, beta = 1
    (eq. 4-1, 4-2).  Decoupling sets lambda_t = lambda_w, so lambda_w K = D_p and
    F_s = Q + F_p."""
    L, Dp, Ds, phi = 2.0, 1e-3, 1e-3, 1.0
    dx = L / N
    dt = dx / c
    coef = oracle.GivenCoefficients(lambda S: Dp + 0 * S, lambda S: Dp + 0 * S)
    bcf = [("abb", lambda x, y, z, t: 1.0 + np.sin(np.pi * x) * np.sin(np.pi * y))] * 4
    bcg = [("abb", lambda x, y, z, t: t * np.sin(np.pi * x) * np.sin(np.pi * y))] * 4
    s = oracle.Solver("D2Q9", (N, N), beta=1.0, Ds=Ds, coef=coef, bc_f=bcf, bc_g=bcg, dx=dx, dt=dt, m=1)
    X, Y = s.X, s.Y
    ss = np.sin(np.pi * X) * np.sin(np.pi * Y)
    Fp = 2 * Dp * np.pi ** 2 * ss

    def sources(t):
        Q = (2 * Ds * np.pi ** 2 * t + phi) * ss
        return Fp, Q + Fp

    s.set_fields(1.0, phi, *sources(0.0))
    dP = np.stack([np.pi * np.cos(np.pi * X) * np.sin(np.pi * Y), np.pi * np.sin(np.pi * X) * np.cos(np.pi * Y), 0 * X])
    s.set_state(1.0 + ss, 0 * ss, dP0=dP, dS0=np.zeros_like(dP))
    iters = [s.step(tol, max_iters, sources=sources) for _ in range(int(round(T / dt)))]
    s.set_sources(*sources(s.t))
    s.update_coefficients()
    iters.append(s.pressure_solve(tol, max_iters)[0])
    u = s.velocity()
    if out is not None:
        out.update(iters=iters, solver=s)
    ua = -Dp * dP
    return dict(EP=rel_l1(1.0 + ss, s.pressure()), Eux=rel_l1(ua[0], u[0]), Euy=rel_l1(ua[1], u[1]),
                ES=rel_l1(s.t * ss, s.saturation()))


def example2(N, c=10.0, T=0.2, phi=1.0, beta=1.0, tol=1e-12, max_iters=2000000, out=None):
    """Example 2: coupled problem on [0,1]^2 with D_p = 1/(0.5 - 0.2 S), D_s = 0.01,
    f_w = S, lambda_w K = f_w D_p, F_p = 0 (eq. 4-4, 4-5)."""
    L, Ds = 1.0, 0.01
    dx = L / N
    dt = dx / c
    coef = oracle.GivenCoefficients(lambda S: 1.0 / (0.5 - 0.2 * S), lambda S: S / (0.5 - 0.2 * S))
    th = lambda x, y, t: np.pi * (x + y - 2 * t)
    Pex = lambda x, y, z, t: -np.cos(th(x, y, t)) / (5 * np.pi) - (x + y) / 2
    Sex = lambda x, y, z, t: np.sin(th(x, y, t))
    s = oracle.Solver("D2Q9", (N, N), beta=beta, Ds=Ds, coef=coef, bc_f=[("abb", Pex)] * 4,
                      bc_g=[("abb", Sex)] * 4, dx=dx, dt=dt, m=1)
    X, Y = s.X, s.Y

    def sources(t):
        return 0.0, 2 * np.pi ** 2 * Ds * np.sin(th(X, Y, t)) + 2 * np.pi * (1 - phi) * np.cos(th(X, Y, t))

    s.set_fields(1.0, phi, *sources(0.0))
    S0 = Sex(X, Y, 0, 0.0)
    gp = S0 / 5 - 0.5
    gs = np.pi * np.cos(th(X, Y, 0.0))
    s.set_state(Pex(X, Y, 0, 0.0), S0, dP0=np.stack([gp, gp, 0 * X]), dS0=np.stack([gs, gs, 0 * X]))
    iters = [s.step(tol, max_iters, sources=sources) for _ in range(int(round(T / dt)))]
    s.set_sources(*sources(s.t))
    s.update_coefficients()
    iters.append(s.pressure_solve(tol, max_iters)[0])
    u = s.velocity()
    if out is not None:
        out.update(iters=iters, solver=s)
    one = np.ones_like(X)
    return dict(EP=rel_l1(Pex(X, Y, 0, s.t), s.pressure()), Eux=rel_l1(one, u[0]), Euy=rel_l1(one, u[1]),
                ES=rel_l1(Sex(X, Y, 0, s.t), s.saturation()))


def example2_saturation(N, c=10.0, T=0.2, phi=1.0, beta=1.0, compensate=False):
    """The saturation lattice of Example 2 alone, driven by the exact pressure.

    Before every saturation step the pressure populations are set to the
    first-order Chapman-Enskog state of the exact P (App. A), f_i = w_i P -
    tau_f dt w_i c_i . grad P, whose local gradient eq. (3-10a) is the exact
    grad P; everything else is the oracle's own saturation step.  This
    isolates the error of eq. (3-2) from that of the pressure solve.

    compensate=True subtracts from F_s the term by which the scheme's
    modified equation differs from eq. (2-18) at fixed c: the collision with
    the gamma term of eq. (3-2) is BGK towards g^eq + w_i c_i . J / c_s^2
    with J = -lambda_w K grad P, whose first moment J puts
    (tau_g - 1/2) dt div(dJ/dt) = D_s / (beta c_s^2) div(dJ/dt) into the
    recovered equation.  For Example 2, J = S (1, 1) and
    div(dJ/dt) = 4 pi^2 sin(pi (x + y - 2t)).
    Returns the global relative L1 error of S at T.
    """
    L, Ds = 1.0, 0.01
    dx = L / N
    dt = dx / c
    coef = oracle.GivenCoefficients(lambda S: 1.0 / (0.5 - 0.2 * S), lambda S: S / (0.5 - 0.2 * S))
    th = lambda x, y, t: np.pi * (x + y - 2 * t)
    Pex = lambda x, y, z, t: -np.cos(th(x, y, t)) / (5 * np.pi) - (x + y) / 2
    Sex = lambda x, y, z, t: np.sin(th(x, y, t))
    s = oracle.Solver("D2Q9", (N, N), beta=beta, Ds=Ds, coef=coef, bc_f=[("abb", Pex)] * 4,
                      bc_g=[("abb", Sex)] * 4, dx=dx, dt=dt, m=1)
    X, Y = s.X, s.Y
    k_comp = Ds / (beta * s.cs2) if compensate else 0.0

    def sources(t):
        Fs = 2 * np.pi ** 2 * Ds * np.sin(th(X, Y, t)) + 2 * np.pi * (1 - phi) * np.cos(th(X, Y, t))
        return 0.0, Fs - k_comp * 4 * np.pi ** 2 * np.sin(th(X, Y, t))

    s.set_fields(1.0, phi, *sources(0.0))
    S0 = Sex(X, Y, 0, 0.0)
    gp = S0 / 5 - 0.5
    gs = np.pi * np.cos(th(X, Y, 0.0))
    s.set_state(Pex(X, Y, 0, 0.0), S0, dP0=np.stack([gp, gp, 0 * X]), dS0=np.stack([gs, gs, 0 * X]))
    for _ in range(int(round(T / dt))):
        s.set_sources(*sources(s.t))
        s.update_coefficients()
        gpx = np.sin(th(X, Y, s.t)) / 5 - 0.5
        f = s.feq(Pex(X, Y, 0, s.t))
        for i in range(1, s.lat.Q):
            ci = s._ev(i)
            f[i] = f[i] - s.tau_f * dt * s.lat.w[i] * (ci[0] + ci[1]) * gpx
        s.f = f
        s.saturation_step()
    s.set_sources(*sources(s.t))
    return rel_l1(Sex(X, Y, 0, s.t), s.saturation())
