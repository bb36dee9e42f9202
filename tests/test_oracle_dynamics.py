"""Pins of the oracle's dynamics beyond one time-invariant linear model
(Sec. IV-A eq. system_eqn, s_{t+1} = s_t + f(s_t, u_t); Sec. IV-B, one SQP
step of the trajectory problem per ADMM iteration):

- the trajectory QP with one linear model per step against the full KKT
  system of the LQ problem, written here;
- the nonlinear bicycle and quadrotor steps and their complex-step
  Jacobians against central differences, closed forms of the motions
  (straight line, constant turn, hover, free fall, yawed hover) and the
  hover / straight-line linear models of the workloads (written
  independently as the textbook linearisations);
- the SQP iteration without obstacles against scipy's SLSQP on the
  nonlinear optimal-control problem (a small horizon), whose model is the
  bicycle written here in numpy;
- per-scenario models: scenarios stay separable and select_scenarios keeps
  each scenario's own models."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
import workloads


def dense_kkt_tv(A, B, c, x0, H, h, Q_u):
    """Full KKT system of the LQ problem with per-step models A[t], B[t], c[t]
    in (x_1..x_N, u_0..u_{N-1})."""
    N, n_s = h.shape
    n_u = B.shape[2]
    nx, nu = N * n_s, N * n_u
    nv = nx + nu
    P = np.zeros((nv, nv))
    q = np.zeros(nv)
    for t in range(N):
        P[t * n_s:(t + 1) * n_s, t * n_s:(t + 1) * n_s] = H[t]
        q[t * n_s:(t + 1) * n_s] = h[t]
        P[nx + t * n_u:nx + (t + 1) * n_u, nx + t * n_u:nx + (t + 1) * n_u] = 2 * Q_u
    E = np.zeros((nx, nv))
    e = np.zeros(nx)
    for t in range(N):
        # x_{t+1} - A_t x_t - B_t u_t = c_t
        E[t * n_s:(t + 1) * n_s, t * n_s:(t + 1) * n_s] = np.eye(n_s)
        E[t * n_s:(t + 1) * n_s, nx + t * n_u:nx + (t + 1) * n_u] = -B[t]
        if t == 0:
            e[:n_s] = A[0] @ x0 + c[0]
        else:
            E[t * n_s:(t + 1) * n_s, (t - 1) * n_s:t * n_s] = -A[t]
            e[t * n_s:(t + 1) * n_s] = c[t]
    KKT = np.block([[P, E.T], [E, np.zeros((nx, nx))]])
    sol = np.linalg.solve(KKT, np.r_[-q, e])
    return np.vstack([x0, sol[:nx].reshape(N, n_s)]), sol[nx:nv].reshape(N, n_u)


@pytest.mark.parametrize("n_s,n_u", [(4, 2), (12, 4)])
def test_time_varying_traj_qp_vs_dense_kkt(n_s, n_u):
    rng = np.random.default_rng(11)
    N = 10
    for _ in range(3):
        A = np.eye(n_s)[None] + 0.1 * rng.normal(size=(N, n_s, n_s))
        B = 0.2 * rng.normal(size=(N, n_s, n_u))
        c = 0.1 * rng.normal(size=(N, n_s))
        H = np.array([(lambda M: M @ M.T + 0.5 * np.eye(n_s))(rng.normal(size=(n_s, n_s))) for _ in range(N)])
        h = rng.normal(size=(N, n_s))
        Qm = rng.normal(size=(n_u, n_u))
        Qu = Qm @ Qm.T + 0.2 * np.eye(n_u)
        x0 = rng.normal(size=n_s)
        x, u = oracle.traj_qp(A, B, c, x0, H, h, Qu)
        xd, ud = dense_kkt_tv(A, B, c, x0, H, h, Qu)
        assert np.allclose(x, xd, atol=1e-9, rtol=1e-9)
        assert np.allclose(u, ud, atol=1e-9, rtol=1e-9)
        # the time-varying path with all models equal is the time-invariant one
        x1, u1 = oracle.traj_qp(np.repeat(A[:1], N, 0), np.repeat(B[:1], N, 0), np.repeat(c[:1], N, 0),
                                x0, H, h, Qu)
        x2, u2 = oracle.traj_qp(A[0], B[0], c[0], x0, H, h, Qu)
        assert np.allclose(x1, x2, atol=1e-12) and np.allclose(u1, u2, atol=1e-12)


def _model_problem(model):
    p = workloads.make("c2sqp" if model == 1 else "c3sqp")
    return oracle.Problem(p), p


@pytest.mark.parametrize("model", [1, 2])
def test_complex_step_jacobians_vs_central_differences(model):
    P, p = _model_problem(model)
    rng = np.random.default_rng(model)
    n_s, n_u = p["n_s"], p["n_u"]
    for _ in range(5):
        s = rng.normal(size=n_s) * (0.3 if model == 2 else 1.0)
        u = rng.normal(size=n_u) * 0.2
        F, A, B = P.model_step(s, u)
        h = 1e-6
        for j in range(n_s + n_u):
            e = np.zeros(n_s + n_u)
            e[j] = h
            Fp = P.model_step(s + e[:n_s], u + e[n_s:])[0]
            Fm = P.model_step(s - e[:n_s], u - e[n_s:])[0]
            col = (Fp - Fm) / (2 * h)
            ref = A[:, j] if j < n_s else B[:, j - n_s]
            assert np.allclose(ref, col, rtol=1e-6, atol=1e-8), j


def test_bicycle_closed_forms():
    P, p = _model_problem(1)
    dt, L = p["model_par"]
    # straight line: no steering, no acceleration
    s = np.array([3.0, -2.0, 0.4, 7.0])
    F, A, B = P.model_step(s, np.zeros(2))
    assert np.allclose(F, [3.0 + dt * 7.0 * np.cos(0.4), -2.0 + dt * 7.0 * np.sin(0.4), 0.4, 7.0], atol=1e-14)
    # constant steering: yaw advances by v tan(delta) / L per unit time; acceleration adds dt a
    F, _, _ = P.model_step(s, np.array([1.5, 0.1]))
    assert F[2] == pytest.approx(0.4 + dt * 7.0 * np.tan(0.1) / L, abs=1e-14)
    assert F[3] == pytest.approx(7.0 + dt * 1.5, abs=1e-14)
    # the straight-reference linearisation of the workloads
    v = 20.0
    _, A, B = P.model_step(np.array([0.0, 0.0, 0.0, v]), np.zeros(2))
    A0, B0, c0 = workloads.bicycle_model(v, dt, L)
    assert np.allclose(A, A0, atol=1e-13) and np.allclose(B, B0, atol=1e-13)


def test_quadrotor_closed_forms():
    P, p = _model_problem(2)
    dt, m, Jx, Jy, Jz, g = p["model_par"][:6]
    s = np.zeros(12)
    s[:3] = [1.0, 2.0, 3.0]
    # hover is a fixed point
    F, A, B = P.model_step(s, np.zeros(4))
    assert np.allclose(F, s, atol=1e-14)
    # the hover linearisation of the workloads
    A0, B0, _ = workloads.quadrotor_model(dt, m, (Jx, Jy, Jz), g)
    assert np.allclose(A, A0, atol=1e-12) and np.allclose(B, B0, atol=1e-12)
    # free fall: thrust change -m g cancels gravity's support
    F, _, _ = P.model_step(s, np.array([-m * g, 0, 0, 0]))
    assert F[5] == pytest.approx(-dt * g, abs=1e-13)
    # yaw does not tilt the thrust: a yawed hover stays a fixed point
    s2 = s.copy()
    s2[8] = 0.7
    assert np.allclose(P.model_step(s2, np.zeros(4))[0], s2, atol=1e-13)
    # a spin about the body z axis of a diagonal inertia keeps its rate
    s3 = s.copy()
    s3[11] = 2.0
    F, _, _ = P.model_step(s3, np.zeros(4))
    assert F[11] == pytest.approx(2.0, abs=1e-14) and F[8] == pytest.approx(dt * 2.0, abs=1e-14)
    # a pitch theta tilts the thrust toward +x: v_x' = g sin(theta), v_z' = g cos(theta) - g
    s4 = s.copy()
    s4[7] = 0.2
    F, _, _ = P.model_step(s4, np.zeros(4))
    assert F[3] == pytest.approx(dt * g * np.sin(0.2), abs=1e-13)
    assert F[5] == pytest.approx(dt * (g * np.cos(0.2) - g), abs=1e-13)


def _bicycle_np(x, u, dt, L):
    return np.array([x[0] + dt * x[3] * np.cos(x[2]), x[1] + dt * x[3] * np.sin(x[2]),
                     x[2] + dt * x[3] * np.tan(u[1]) / L, x[3] + dt * u[0]])


def test_sqp_without_obstacles_reaches_the_nonlinear_optimum():
    """No obstacles: each ADMM iteration is one SQP step of the nonlinear
    tracking problem; its fixed point is the optimum of that problem, found
    independently by SLSQP (Sec. IV-B: one QP per iteration)."""
    N, dt, L = 6, 0.1, 2.7
    p = workloads.with_obstacles(workloads.make("c1"), [[]])
    p = dict(p)
    p["N"] = N
    # a reference that turns: the straight-line linearisation is not exact
    xr = np.zeros((1, N + 1, 4))
    x = np.array([0.0, 0.0, 0.0, 10.0])
    for t in range(N + 1):
        xr[0, t] = x
        x = _bicycle_np(x, (0.5, 0.15), dt, L)
    p.update(x_ref=xr, x0=xr[:, 0].copy() + np.array([[0.0, 0.3, 0.05, 0.0]]),
             model=workloads.MODEL_BICYCLE, model_par=np.array([dt, L]), eps_pri=-1.0, eps_dual=-1.0)
    A0, B0, c0 = workloads.bicycle_model(10.0, dt, L)
    p.update(A_dyn=A0, B_dyn=B0, c_dyn=c0)
    P = oracle.Problem(p)
    st = P.init_state()
    P.run(st, 40)
    Qs, Qu = p["Q_s"], p["Q_u"]
    x0 = p["x0"][0]

    def unpack(z):
        u = z.reshape(N, 2)
        xs = [x0]
        for t in range(N):
            xs.append(_bicycle_np(xs[-1], u[t], dt, L))
        return np.array(xs), u

    def cost(z):
        xs, u = unpack(z)
        e = xs[1:] - xr[0, 1:]
        return np.einsum("ti,ij,tj->", e, Qs, e) + np.einsum("ti,ij,tj->", u, Qu, u)

    res = minimize(cost, np.zeros(2 * N), method="SLSQP", options=dict(ftol=1e-14, maxiter=500))
    xs, us = unpack(res.x)
    assert np.allclose(st["u"][0], us, atol=1e-5)
    assert np.allclose(st["x"][0], xs, atol=1e-5)
    # the iterate satisfies the nonlinear dynamics (the SQP defects are closed)
    for t in range(N):
        assert np.allclose(_bicycle_np(st["x"][0, t], st["u"][0, t], dt, L), st["x"][0, t + 1], atol=1e-9)


def test_per_scenario_models_are_separable():
    """The time-varying workload (one model per scenario and step): running
    scenarios together or alone gives the same iterates, and select_scenarios
    keeps each scenario's own models."""
    p = workloads.make("c2tv")
    P = oracle.Problem(p)
    st = P.init_state()
    P.run(st, 5)
    for s in (1, 3):
        q = workloads.select_scenarios(p, [s])
        Q = oracle.Problem(q)
        sq = Q.init_state()
        Q.run(sq, 5)
        assert np.allclose(sq["x"][0], st["x"][s], atol=1e-10, rtol=0)
        N = p["N"]
        assert np.array_equal(q["A_dyn"], p["A_dyn"][s * N:(s + 1) * N])
