"""Pins of the dual-EnKF oracle on the inlet-forced Burgers case: the open
prolongation (one-sided cubic stencils) reproduces cubics and inverts
injection, uniform flow is an exact steady state, the scheme converges at
second order under grid refinement, the parameter update equals the
textbook ensemble Kalman update written with an explicit inverse, the
random walk has the requested moments, and a short dual MEnKF run moves
the amplitude estimate from its prior toward the truth."""

import numpy as np

from oracle import dual, enkf, rng
from synthetic import configs, fields


def test_open_prolongation_reproduces_cubics_and_inverts_injection():
    for nc, r in ((12, 4), (9, 3), (8, 1), (16, 8)):
        P = dual.prolong_matrix_open(nc, r)
        np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-13)
        X = np.arange(nc, dtype=np.float64)          # coarse coordinate in coarse-node units
        xf = np.arange(nc * r) / r
        for deg in range(4):
            np.testing.assert_allclose(P @ X ** deg, xf ** deg, rtol=0, atol=1e-9 * max(1.0, nc ** deg))
        # injection after prolongation is the identity on the coarse grid
        np.testing.assert_allclose(P[::r], np.eye(nc), atol=1e-14)
        xc = np.random.default_rng(nc).standard_normal((3, nc))
        np.testing.assert_allclose(dual.restrict_open(dual.prolong_open(xc, r), r), xc, atol=1e-13)


def test_uniform_flow_is_a_steady_state():
    cfg = configs.inlet_burgers(nx=200)
    u = fields.inlet_uniform(cfg)
    out, prev = dual.inlet_forecast(u, 0.0, 500, cfg.dt, np.array([0.0, 0.7]), cfg.nu, cfg.length / cfg.nx,
                                    cfg.u0, cfg.omega)
    np.testing.assert_array_equal(out, u)
    np.testing.assert_array_equal(prev, u)


def test_second_order_under_refinement():
    """Self-convergence of the inlet wave at t = 0.5 on n = 100 ... 800 cells
    (common nodes x = 0.1 k): successive differences shrink by 4 per halving.
    The viscosity is raised to 0.05 so that the front launched by the inlet
    at t = 0 is resolved on the coarsest grid and the asymptotic rate shows."""
    L, nu, u0, om = 10.0, 0.05, 1.0, np.pi
    th = np.array([0.2, 0.0])
    T, dt = 0.5, 5e-5

    def run(n):
        u = np.full((1, n), u0)
        out, _ = dual.inlet_forecast(u, 0.0, int(round(T / dt)), dt, th, nu, L / n, u0, om)
        return out[0, ::n // 100][:10]
    s = [run(n) for n in (100, 200, 400, 800)]
    d = [np.abs(s[i] - s[i + 1]).max() for i in range(3)]
    orders = [np.log2(d[i] / d[i + 1]) for i in range(2)]
    assert all(1.85 < o < 2.2 for o in orders), (d, orders)


def test_parameter_update_is_the_ensemble_kalman_update():
    """theta^a = theta^f + Theta Y^T (Y Y^T + R)^-1 (y^o + eps - y^f), with an
    explicit inverse, for a nonlinear map of the parameters to probes."""
    g = np.random.default_rng(3)
    N, P, Ny, sig = 30, 2, 7, 0.05
    theta_f = g.standard_normal((N, P)) * 0.1 + np.array([0.1, 0.3])
    A = g.standard_normal((Ny, P))
    yf = np.tanh(theta_f @ A.T)                       # (N, Ny), nonlinear in theta
    yo = g.standard_normal(Ny) * 0.1
    eps = sig * g.standard_normal((N, Ny))
    # enkf.analysis works on states; use the observations themselves as the state
    xs = yf[:, None, :]
    res = enkf.analysis(xs, yf.mean(axis=0)[None, :], yo, eps, lambda x: x[..., 0, :], sig)
    got = dual.param_update(theta_f, res["Z"])
    Th = (theta_f - theta_f.mean(0)) / np.sqrt(N - 1)
    Y = (yf - yf.mean(0)) / np.sqrt(N - 1)
    K = Th.T @ Y @ np.linalg.inv(Y.T @ Y + sig ** 2 * np.eye(Ny))
    want = theta_f + (K @ (yo[None, :] + eps - yf).T).T
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_random_walk_moments_and_independence_from_observation_draws():
    tau = dual.param_perturbations(7, 3, 20000, [0.01, 0.002])
    assert abs(tau[:, 0].mean()) < 3 * 0.01 / np.sqrt(20000)
    assert abs(tau[:, 0].std() / 0.01 - 1) < 0.03
    assert abs(tau[:, 1].std() / 0.002 - 1) < 0.03
    eps = rng.perturbations(7, 3, 20000, 2, 1.0)
    assert abs(np.corrcoef(tau[:, 0], eps[:, 0])[0, 1]) < 0.05


def test_short_dual_run_moves_the_amplitude_toward_the_truth():
    cfg = configs.inlet_burgers(nx=200, ratio=2, n_members=40, n_probes=20, n_obs=30)
    idx, _ = fields.probes_for(cfg)
    hf = cfg.length / cfg.nx
    truth = fields.inlet_uniform(cfg)
    truth, _ = dual.inlet_forecast(truth, 0.0, 5000, cfg.dt, np.array(cfg.theta_true), cfg.nu, hf, cfg.u0, cfg.omega)
    st = dual.DualState(fine=fields.inlet_uniform(cfg), members=fields.inlet_uniform(cfg, "coarse", cfg.n_members),
                        theta=fields.inlet_theta_ics(cfg), t=1.0)
    # a short free spin-up of the model side from t = 0 to 1
    st.fine, _ = dual.inlet_forecast(st.fine, 0.0, 5000, cfg.dt, st.theta.mean(0), cfg.nu, hf, cfg.u0, cfg.omega)
    st.members, _ = dual.inlet_forecast(st.members, 0.0, 5000, cfg.dt, st.theta, cfg.nu, cfg.length / cfg.nxc,
                                        cfg.u0, cfg.omega)
    t = 1.0
    for c in range(1, 61):
        truth, _ = dual.inlet_forecast(truth, t, cfg.n_obs, cfg.dt, np.array(cfg.theta_true), cfg.nu, hf, cfg.u0,
                                       cfg.omega)
        t += cfg.n_obs * cfg.dt
        y = truth[0, idx] + fields.obs_noise(cfg, c)
        st, theta_bar = dual.dual_cycle(cfg, st, y, idx, n_sweeps=1)
    # prior (0, 0.3), truth (0.2, 0): the amplitude is found within 60
    # cycles, the phase has moved most of the way
    assert abs(theta_bar[0] - 0.2) < 0.05, theta_bar
    assert theta_bar[1] < 0.2, theta_bar


def test_correction_keeps_the_inlet_and_sweeps_solve_the_implicit_system():
    cfg = configs.inlet_burgers(nx=200, ratio=4, n_members=8, n_probes=20)
    hf = cfg.length / cfg.nx
    g = np.random.default_rng(5)
    xf = 1.0 + 0.1 * np.sin(np.arange(cfg.nx) * hf)[None, :] + 0.01 * g.standard_normal((1, cfg.nx))
    delta = 0.05 * g.standard_normal((1, cfg.nxc))
    x = dual.correct_open(xf, delta, cfg.ratio)
    assert x[0, 0] == xf[0, 0]
    np.testing.assert_allclose(x[0, 1:], xf[0, 1:] + dual.prolong_open(delta, cfg.ratio)[0, 1:], atol=0)
    xprev = xf - 0.001
    y = dual.smooth_open(x, xprev, cfg, 0, 0.5)
    np.testing.assert_array_equal(y, x)
    # undamped Jacobi converges to the implicit-Euler solution at the interior
    y = dual.smooth_open(x, xprev, cfg, 400, 1.0)      # (1, n): one state of one field
    r = xprev + cfg.dt * dual._rhs(y, cfg.nu, hf) - y
    assert np.abs(r[0, 1:-1]).max() < 1e-13
    assert y[0, 0] == x[0, 0]
    assert y[0, -1] == 2.0 * y[0, -2] - y[0, -3]


# ------------------------------------------------------------------ the paper's first-order scheme
def _psi_matrix(u0, dt, nu, h):
    """Psi = I - dt L_{u0} of the implicit-Euler step at the interior nodes,
    with the convective coefficient frozen at u0, written out densely:
    (Psi x)_i = x_i - dt (-u0_i (x_{i+1} - x_{i-1}) / 2h + nu (x_{i+1} - 2 x_i + x_{i-1}) / h^2)."""
    n = u0.shape[-1]
    P = np.eye(n)
    for i in range(1, n - 1):
        P[i, i - 1] += -dt * (u0[i] / (2 * h) + nu / h ** 2)
        P[i, i] += dt * 2 * nu / h ** 2
        P[i, i + 1] += -dt * (-u0[i] / (2 * h) + nu / h ** 2)
    return P


def test_first_order_analysis_step_is_one_jacobi_iteration():
    """The last step of a first-order window is x^1 = x^0 + diag(Psi)^-1 (c - Psi x^0)
    at the interior nodes, with c = x^0 = x_{k-1}, the inlet value at t_k and
    the outlet extrapolated; the steps before it are forward Euler."""
    n, dt, nu, h, u0, om = 14, 2e-3, 0.02, 0.1, 1.0, 2 * np.pi
    th = np.array([0.3, 0.4])
    x0 = 1.0 + 0.2 * np.sin(np.arange(n) * 0.7)
    x0[0] = dual.inlet_value(0.0, th, u0, om)
    out, prev = dual.inlet_forecast_first_order(x0[None], 0.0, 1, dt, th, nu, h, u0, om)
    P = _psi_matrix(x0, dt, nu, h)
    jac = x0 + (x0 - P @ x0) / np.diag(P)
    np.testing.assert_allclose(out[0, 1:-1], jac[1:-1], rtol=0, atol=1e-14)
    assert out[0, 0] == dual.inlet_value(dt, th, u0, om)
    assert out[0, -1] == 2 * out[0, -2] - out[0, -3]
    np.testing.assert_array_equal(prev[0], x0)
    # two steps: a forward-Euler step (L from the explicit definition) then the Jacobi step
    out2, prev2 = dual.inlet_forecast_first_order(x0[None], 0.0, 2, dt, th, nu, h, u0, om)
    fe = x0 - (P - np.eye(n)) @ x0                                 # x0 + dt L x0 = x0 - (Psi - I) x0
    fe[0] = dual.inlet_value(dt, th, u0, om)
    fe[-1] = 2 * fe[-2] - fe[-3]
    np.testing.assert_allclose(prev2[0], fe, rtol=0, atol=1e-14)
    P2 = _psi_matrix(fe, dt, nu, h)
    jac2 = fe + (fe - P2 @ fe) / np.diag(P2)
    np.testing.assert_allclose(out2[0, 1:-1], jac2[1:-1], rtol=0, atol=1e-14)


def test_jacobi_iterated_solves_the_implicit_step():
    """Repeating the splitting (coefficients re-frozen at each iterate)
    converges to the solution of the nonlinear implicit-Euler step, which a
    dense Newton solve of x - dt L(x) = c finds independently: the single
    iteration the scheme takes is the first of a convergent sequence."""
    n, dt, nu, h = 16, 5e-3, 0.05, 0.1
    c = 1.0 + 0.3 * np.cos(np.arange(n) * 0.5)
    x = c.copy()
    for _ in range(200):
        P = _psi_matrix(x, dt, nu, h)
        x[1:-1] = (x + (c - P @ x) / np.diag(P))[1:-1]
    z = c.copy()
    for _ in range(30):                        # Newton on the interior nodes, boundary values fixed at c
        F = z - c
        F[1:-1] = z[1:-1] - dt * (-z[1:-1] * (z[2:] - z[:-2]) / (2 * h) + nu * (z[2:] - 2 * z[1:-1] + z[:-2]) / h ** 2) - c[1:-1]
        J = np.eye(n)
        for i in range(1, n - 1):
            J[i, i - 1] = -dt * (z[i] / (2 * h) + nu / h ** 2)
            J[i, i] = 1 + dt * ((z[i + 1] - z[i - 1]) / (2 * h) + 2 * nu / h ** 2)
            J[i, i + 1] = -dt * (-z[i] / (2 * h) + nu / h ** 2)
        z = z - np.linalg.solve(J, F)
    np.testing.assert_allclose(x, z, rtol=0, atol=1e-12)


def test_first_order_scheme_converges_at_first_order_in_time():
    """The explicit steps of the first-order scheme: halving dt halves the
    error at a fixed time against a much finer step (one Jacobi step at
    the end of each window of 10 steps)."""
    L, n, nu, u0, om = 10.0, 200, 0.02, 1.0, 2 * np.pi
    th = np.array([0.2, 0.0])
    T = 0.4

    def run(dt):
        u = np.full((1, 1, n), u0)
        t = 0.0
        steps = int(round(T / dt))
        for w in range(steps // 10):
            u, _ = dual.inlet_forecast_first_order(u, t, 10, dt, th, nu, L / n, u0, om)
            t += 10 * dt
        return u[0, 0]
    ref = run(2.5e-5)
    e = [np.abs(run(dt) - ref).max() for dt in (1e-3, 5e-4, 2.5e-4)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(0.85 < o < 1.25 for o in orders), (e, orders)


def test_first_order_uniform_flow_is_steady():
    cfg = configs.inlet_burgers(nx=200, time_scheme="first_order")
    u = fields.inlet_uniform(cfg)
    out, prev = dual.inlet_forecast_first_order(u, 0.0, 30, cfg.dt, np.array([0.0, 0.7]), cfg.nu,
                                                cfg.length / cfg.nx, cfg.u0, cfg.omega)
    np.testing.assert_array_equal(out, u)
