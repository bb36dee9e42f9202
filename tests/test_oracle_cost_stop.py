"""Pins of the oracle's tracking cost (Sec. IV-A eq. navigation_cost), of its
x0 gradient through unrolled iterations, and of the stopping-test sums
(Sec. IV-B), each against something other than the oracle itself:

- the obstacle-free ADMM iterate is the LQ optimum, whose cost is the LQ value
  function V_0(x0) = x0^T P_0 x0 + 2 q_0^T x0 + r_0 of a Riccati recursion
  written here from the textbook (the oracle solves its LQ problems by a
  condensed Cholesky solve instead), and whose x0 gradient is 2 P_0 x0 + 2 q_0;
- r_pri and r_dual equal the sums of squared changes of (zeta, xi) and of the
  lambda and mu rows (gamma excluded), formed here from the iterates the
  oracle hands back before and after one iteration.
"""
import numpy as np
import pytest

import oracle
import workloads


def value_function(A, B, c, Q_s, Q_u, x_ref, N):
    """Cost-to-go V_t(x) = x^T P_t x + 2 q_t^T x + r_t of
    F = sum_{t=1..N} (x_t - xr_t)^T Q_s (x_t - xr_t) + sum_{t=0..N-1} u_t^T Q_u u_t
    subject to x_{t+1} = A x_t + B u_t + c, by the backward recursion
    V_t(x) = [t >= 1] (x - xr_t)^T Q_s (x - xr_t) + min_u { u^T Q_u u + V_{t+1}(A x + B u + c) }.
    Returns (P_0, q_0, r_0)."""
    xr = x_ref[N]
    P = Q_s.copy()
    q = -Q_s @ xr
    r = xr @ Q_s @ xr
    for t in range(N - 1, -1, -1):
        # min over u of u^T Q_u u + (A x + B u + c)^T P (A x + B u + c) + 2 q^T (A x + B u + c) + r
        S = Q_u + B.T @ P @ B
        L = B.T @ P @ A                      # cross term u^T L x (twice)
        l = B.T @ (P @ c + q)                # linear term in u (twice)
        Sinv = np.linalg.inv(S)
        Pn = A.T @ P @ A - L.T @ Sinv @ L
        qn = A.T @ (P @ c + q) - L.T @ Sinv @ l
        rn = c @ P @ c + 2 * q @ c + r - l @ Sinv @ l
        if t >= 1:
            xr = x_ref[t]
            Pn = Pn + Q_s
            qn = qn - Q_s @ xr
            rn = rn + xr @ Q_s @ xr
        P, q, r = 0.5 * (Pn + Pn.T), qn, rn
    return P, q, r


def obstacle_free(name, seed_shift):
    """The configuration's robot, model and cost with no obstacles, an initial
    state off the reference and a bent reference, so that every term of F
    (states t = 1..N, inputs t = 0..N-1) is non-zero."""
    p = workloads.with_obstacles(workloads.make(name), [[]])
    rng = np.random.default_rng(seed_shift)
    n_s, N = p["n_s"], p["N"]
    p["x_ref"] = p["x_ref"].copy()
    p["x_ref"][0, :, :] += 0.3 * rng.normal(size=(N + 1, n_s)).cumsum(0) / np.sqrt(N)
    p["x0"] = p["x_ref"][:, 0, :] + 0.5 * rng.normal(size=(1, n_s))
    return p


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_cost_of_lq_optimum_is_value_function(name):
    p = obstacle_free(name, 3)
    P = oracle.Problem(p)
    st = P.init_state()
    F = P.cost(st["x"], st["u"], 0)
    Pm, q, r = value_function(p["A_dyn"], p["B_dyn"], p["c_dyn"], p["Q_s"], p["Q_u"], p["x_ref"][0], p["N"])
    x0 = p["x0"][0]
    V = x0 @ Pm @ x0 + 2 * q @ x0 + r
    assert F > 1.0
    assert abs(F - V) <= 1e-9 * V
    # the ADMM iteration leaves the obstacle-free optimum where it is
    P.run(st, 3)
    assert abs(P.cost(st["x"], st["u"], 0) - V) <= 1e-9 * V


@pytest.mark.parametrize("name,K", [("c1", 1), ("c1", 4), ("c3", 2)])
def test_x0_gradient_is_value_function_gradient(name, K):
    p = obstacle_free(name, 5)
    p["eps_pri"] = p["eps_dual"] = -1.0
    L, gd, gx = oracle.grad_fixed_y0(p, K, np.zeros(0))
    Pm, q, r = value_function(p["A_dyn"], p["B_dyn"], p["c_dyn"], p["Q_s"], p["Q_u"], p["x_ref"][0], p["N"])
    x0 = p["x0"][0]
    g = 2 * Pm @ x0 + 2 * q
    assert abs(L - (x0 @ Pm @ x0 + 2 * q @ x0 + r)) <= 1e-9 * abs(L)
    assert np.linalg.norm(gx[0] - g) <= 1e-8 * np.linalg.norm(g)


def test_value_function_matches_brute_force_cost():
    """The recursion above, checked on its own against the cost of the
    optimum of the dense least-squares problem over the stacked inputs."""
    rng = np.random.default_rng(2)
    n_s, n_u, N = 3, 2, 6
    A = np.eye(n_s) + 0.2 * rng.normal(size=(n_s, n_s))
    B = rng.normal(size=(n_s, n_u))
    c = 0.1 * rng.normal(size=n_s)
    Q_s = np.diag(rng.uniform(0.5, 2.0, n_s))
    Q_u = np.diag(rng.uniform(0.1, 1.0, n_u))
    xr = rng.normal(size=(N + 1, n_s))
    x0 = rng.normal(size=n_s)
    # x_t = Phi_t x0 + sum_k G_{t,k} u_k + e_t: stack and minimise
    Phi = [np.eye(n_s)]
    e = [np.zeros(n_s)]
    for t in range(N):
        Phi.append(A @ Phi[-1])
        e.append(A @ e[-1] + c)
    G = np.zeros((N + 1, n_s, N * n_u))
    for t in range(1, N + 1):
        G[t] = A @ G[t - 1]
        G[t][:, (t - 1) * n_u:t * n_u] += B
    rows, rhs = [], []
    Ls, Lu = np.linalg.cholesky(Q_s).T, np.linalg.cholesky(Q_u).T
    for t in range(1, N + 1):
        rows.append(Ls @ G[t])
        rhs.append(Ls @ (xr[t] - Phi[t] @ x0 - e[t]))
    for t in range(N):
        blk = np.zeros((n_u, N * n_u))
        blk[:, t * n_u:(t + 1) * n_u] = Lu
        rows.append(blk)
        rhs.append(np.zeros(n_u))
    U = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)[0]
    F = 0.0
    for t in range(1, N + 1):
        d = Phi[t] @ x0 + e[t] + G[t] @ U - xr[t]
        F += d @ Q_s @ d
    for t in range(N):
        u = U[t * n_u:(t + 1) * n_u]
        F += u @ Q_u @ u
    Pm, q, r = value_function(A, B, c, Q_s, Q_u, xr, N)
    assert abs(F - (x0 @ Pm @ x0 + 2 * q @ x0 + r)) <= 1e-10 * F


@pytest.mark.parametrize("name,k", [("c1", 0), ("c1", 6), ("c2", 2)])
def test_stop_sums_are_squared_changes(name, k):
    """r_pri = sum (dzeta^2 + |dxi|^2) and r_dual = sum (|dlambda|^2 + |dmu|^2)
    over every pair of the scenario, gamma excluded (Sec. IV-B stopping
    criteria), formed from the iterates before and after one iteration."""
    p = workloads.make(name)
    p["eps_pri"] = p["eps_dual"] = -1.0
    P = oracle.Problem(p)
    st = P.init_state()
    if k:
        P.run(st, k)
    before = {key: v.copy() for key, v in st.items()}
    hist = P.run(st, 1)
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(p)
    N = p["N"]
    dz = st["zeta"] - before["zeta"]
    dxi = st["xi"] - before["xi"]
    dy = st["y"] - before["y"]
    r_pri = (dz ** 2).sum() + (dxi ** 2).sum()
    r_dual = 0.0
    dgam = 0.0
    for b in range(len(sc)):
        blk = dy[yoff[b]:yoff[b] + nrow[b] * N].reshape(nrow[b], N)
        r_dual += (blk[:-1] ** 2).sum()
        dgam += (blk[-1] ** 2).sum()
    assert r_pri > 0 and r_dual > 0
    assert abs(hist["r_pri"][0, 0] - r_pri) <= 1e-12 * max(r_pri, 1.0)
    assert abs(hist["r_dual"][0, 0] - r_dual) <= 1e-12 * max(r_dual, 1.0)
    if dgam > 1e-6 * r_dual:
        # gamma moved in this step, so a sum that included it would differ
        assert abs(hist["r_dual"][0, 0] - (r_dual + dgam)) > 1e-9 * r_dual
