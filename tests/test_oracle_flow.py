"""Pins of the velocity -> source oracle (oracle/flow.py): difference rules
exact on low-degree polynomials, the Navier-Stokes source of polynomial
fields against hand derivatives, second-order convergence to the analytic
pressure gradient of the Taylor vortex, and closed forms of the RANS and
compressible forms."""

import numpy as np

from oracle import flow as Fl


def _grid(shape, spacing):
    """Cell-centre coordinate arrays (x, y[, z]) in storage order."""
    axes = [np.arange(n) * h + 0.3 for n, h in zip(reversed(shape), spacing)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(mesh))


def test_difference_rules_are_exact_on_polynomials():
    sp = (0.5, 0.25, 0.4)
    x, y, z = _grid((5, 6, 7), sp)
    f = 1.0 + 2 * x - 3 * y * y + 0.5 * z * x + 0.7 * z * z
    assert np.allclose(Fl.d1(f, sp[0], 0), 2 + 0.5 * z, atol=1e-12)
    assert np.allclose(Fl.d1(f, sp[1], 1), -6 * y, atol=1e-12)
    assert np.allclose(Fl.d1(f, sp[2], 2), 0.5 * x + 1.4 * z, atol=1e-12)
    c = x ** 3 - 2 * y ** 3 + x * y * z + z ** 3
    assert np.allclose(Fl.d2(c, sp[0], 0), 6 * x, atol=1e-10)
    assert np.allclose(Fl.d2(c, sp[1], 1), -12 * y, atol=1e-10)
    assert np.allclose(Fl.d2(c, sp[2], 2), 6 * z, atol=1e-10)
    # degenerate lengths
    assert np.all(Fl.d1(np.ones((1, 4)), 1.0, 1) == 0)
    assert np.allclose(Fl.d1(np.array([[1.0, 3.0]]), 0.5, 0), 4.0)


def test_navier_stokes_source_of_a_polynomial_field():
    """u = (a y + b x^2, c x + d y), steady and unsteady, against derivatives
    taken by hand: f_i = -rho (dudt_i + u_j du_i/dx_j) + mu lap u_i."""
    sp = (0.2, 0.3)
    x, y = _grid((9, 11), sp)
    a, b, c, d = 0.7, -0.4, 1.3, 0.2
    u = [a * y + b * x * x, c * x + d * y]
    rho, mu = 1.7, 0.05
    dudt = [0.3 * x, -0.1 * np.ones_like(x)]
    f = Fl.ns_source(u, sp, rho, mu, dudt)
    fx = -rho * (dudt[0] + u[0] * (2 * b * x) + u[1] * a) + mu * (2 * b)
    fy = -rho * (dudt[1] + u[0] * c + u[1] * d) + mu * 0.0
    assert np.allclose(f[0], fx, atol=1e-12) and np.allclose(f[1], fy, atol=1e-12)


def test_taylor_vortex_source_converges_at_second_order():
    """The Navier-Stokes source of the decaying Taylor vortex (exact time
    derivative, mu = rho nu) approaches its analytic pressure gradient with
    the grid spacing squared."""
    errs, errs_inviscid = [], []
    for n in (81, 161, 321):
        h = 6.0 / (n - 1)
        u, P, g = Fl.taylor_vortex((n, n), (h, h), t=1.0)
        dudt = Fl.taylor_vortex_dudt((n, n), (h, h), t=1.0)
        scale = np.sqrt(np.mean(g[0] ** 2 + g[1] ** 2))
        rel = lambda f: np.sqrt(np.mean((f[0] - g[0]) ** 2 + (f[1] - g[1]) ** 2)) / scale  # noqa: E731
        errs.append(rel(Fl.ns_source(u, (h, h), rho=1.0, mu=1.0, dudt=dudt)))
        # for this flow the unsteady and viscous terms cancel exactly, so the
        # steady inviscid form converges to the same gradient
        errs_inviscid.append(rel(Fl.ns_source(u, (h, h), rho=1.0, mu=0.0)))
    assert errs[-1] < 5e-3 and errs_inviscid[-1] < 1e-4
    for e in (errs, errs_inviscid):
        for e0, e1 in zip(e, e[1:]):
            assert 3.5 < e0 / e1 < 4.9, e
    # snapshot differences approximate the time derivative at second order too
    n, h = 81, 6.0 / 80
    dt = 1e-3
    up, _, _ = Fl.taylor_vortex((n, n), (h, h), t=1.0 - dt)
    un, _, _ = Fl.taylor_vortex((n, n), (h, h), t=1.0 + dt)
    exact = Fl.taylor_vortex_dudt((n, n), (h, h), t=1.0)
    est = Fl.time_derivative(up, un, dt)
    assert np.max(np.abs(est[0] - exact[0])) < 1e-5 * np.max(np.abs(exact[0]))


def test_rans_source_closed_forms():
    sp = (0.5, 0.5, 0.25)
    x, y, z = _grid((4, 5, 6), sp)
    U = [1.0 + 0.5 * y, 0.2 * np.ones_like(x), -0.3 * x]
    # no stresses: the steady inviscid Navier-Stokes source
    a = Fl.rans_source(U, sp, rho=1.2)
    b = Fl.ns_source(U, sp, rho=1.2, mu=0.0)
    for p, q in zip(a, b):
        assert np.allclose(p, q, atol=1e-13)
    # linear stresses add their exact divergence: R_uu = 2x, R_uv = y, R_vw = 3z
    R = [2 * x, np.zeros_like(x), np.zeros_like(x), y, np.zeros_like(x), 3 * z]
    c = Fl.rans_source(U, sp, rho=1.2, R=R)
    assert np.allclose(c[0] - a[0], -1.2 * (2 + 1), atol=1e-12)
    assert np.allclose(c[1] - a[1], -1.2 * (0 + 3), atol=1e-12)
    assert np.allclose(c[2] - a[2], -1.2 * 0, atol=1e-12)


def test_compressible_source_closed_forms():
    sp = (0.1, 0.1, 0.1)
    gas_R, gamma, T_inf, M_inf, V_inf = 287.0, 1.4, 173.0, 2.0, 520.0
    x, y, z = _grid((5, 6, 7), sp)
    # uniform flow: nothing changes, g = 0
    U = [400.0 * np.ones_like(x), 30.0 * np.ones_like(x), np.zeros_like(x)]
    g = Fl.compressible_source(U, sp, gas_R, gamma, T_inf, M_inf, V_inf)
    assert all(np.allclose(c, 0, atol=1e-14) for c in g)
    # flow along x, linear in x: 1-D closed form with hand derivatives
    U = [300.0 + 50.0 * x, np.zeros_like(x), np.zeros_like(x)]
    T = T_inf * (1 + 0.5 * (gamma - 1) * M_inf ** 2 * (1 - U[0] ** 2 / V_inf ** 2))
    dU2 = 2 * U[0] * 50.0
    dT = T_inf * 0.5 * (gamma - 1) * M_inf ** 2 * (-dU2 / V_inf ** 2)
    gx = -(dU2 - U[0] ** 2 / T * dT) / (gas_R * T) / (1 + U[0] ** 2 / (gas_R * T))
    g = Fl.compressible_source(U, sp, gas_R, gamma, T_inf, M_inf, V_inf)
    assert np.allclose(g[0], gx, rtol=1e-12, atol=1e-14)
    assert np.allclose(g[1], 0, atol=1e-14) and np.allclose(g[2], 0, atol=1e-14)
    # fluid at rest with a normal stress linear in x: diagonal system
    U0 = [np.zeros_like(x)] * 3
    Rxx = 1000.0 + 200.0 * x
    R = [Rxx] + [np.zeros_like(x)] * 5
    T0 = T_inf * (1 + 0.5 * (gamma - 1) * M_inf ** 2)
    g = Fl.compressible_source(U0, sp, gas_R, gamma, T_inf, M_inf, V_inf, R=R)
    assert np.allclose(g[0], -(200.0 / (gas_R * T0)) / (1 + Rxx / (gas_R * T0)), rtol=1e-12)


def test_abc_flow_source_converges_at_second_order():
    """3-D: the decaying ABC flow solves the Navier-Stokes equations with
    P = -rho |u|^2 / 2.  The steady inviscid source and the unsteady viscous
    one (snapshot time derivative, mu = rho nu) both approach -grad(rho
    |u|^2 / 2) (derivatives of u taken by hand: d/dx |u|^2 / 2 = e^{-nu t} B
    (v cos x - w sin x), and cyclically) at second order; dropping the viscous term from the unsteady
    form leaves an O(1) error (the time derivative is then unbalanced)."""
    import synth

    A, B, C = 1.0, np.sqrt(2 / 3), np.sqrt(1 / 3)
    rho, nu, t, dt = 1.3, 0.7, 0.4, 1e-4
    errs, errs_steady = [], []
    for n in (24, 48, 96):
        u, _, sp = synth.abc_velocity((n, n, n), t=t, nu=nu, rho=rho)
        u = [c.numpy() for c in u]
        h = sp[0]
        ax = (np.arange(n) + 0.5) * h
        z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
        d = np.exp(-nu * t)  # the decay factor of the derivatives of u
        g = [-rho * d * B * (u[1] * np.cos(x) - u[2] * np.sin(x)),
             -rho * d * C * (u[2] * np.cos(y) - u[0] * np.sin(y)),
             -rho * d * A * (u[0] * np.cos(z) - u[1] * np.sin(z))]
        scale = np.sqrt(np.mean(sum(c * c for c in g)))
        rel = lambda f: np.sqrt(np.mean(sum((a - b) ** 2 for a, b in zip(f, g)))) / scale  # noqa: E731
        up = [c.numpy() for c in synth.abc_velocity((n, n, n), t=t - dt, nu=nu, rho=rho)[0]]
        un = [c.numpy() for c in synth.abc_velocity((n, n, n), t=t + dt, nu=nu, rho=rho)[0]]
        dudt = Fl.time_derivative(up, un, dt)
        errs.append(rel(Fl.ns_source(u, sp, rho, rho * nu, dudt)))
        errs_steady.append(rel(Fl.ns_source(u, sp, rho, 0.0)))
        if n == 96:
            assert rel(Fl.ns_source(u, sp, rho, 0.0, dudt)) > 0.3
    for e in (errs, errs_steady):
        assert e[-1] < 2e-3, e
        # the one-sided end rules of the viscous term are still above their
        # asymptotic ratio of 4 at these sizes (measured 5.2, 5.0)
        for e0, e1 in zip(e, e[1:]):
            assert 3.5 < e0 / e1 < 5.5, e
