"""Pins of the oracle's trajectory QP (Sec. IV-B eq. ADMM_state_updates, one
SQP QP per iteration), the T/R functions (Sec. IV-A), the multiplier update
(eq. ADMM_residue_updates) and the ADMM loop's special cases."""
import numpy as np
import pytest

import oracle
import workloads


def dense_kkt_lq(A, B, c, x0, H, h, Q_u):
    """Full KKT system of the LQ problem in (x_1..x_N, u_0..u_{N-1})."""
    N, n_s = h.shape
    n_u = B.shape[1]
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
        E[t * n_s:(t + 1) * n_s, t * n_s:(t + 1) * n_s] = np.eye(n_s)
        E[t * n_s:(t + 1) * n_s, nx + t * n_u:nx + (t + 1) * n_u] = -B
        if t == 0:
            e[:n_s] = A @ x0 + c
        else:
            E[t * n_s:(t + 1) * n_s, (t - 1) * n_s:t * n_s] = -A
            e[t * n_s:(t + 1) * n_s] = c
    KKT = np.block([[P, E.T], [E, np.zeros((nx, nx))]])
    sol = np.linalg.solve(KKT, np.r_[-q, e])
    x = np.vstack([x0, sol[:nx].reshape(N, n_s)])
    return x, sol[nx:nv].reshape(N, n_u)


def riccati_lq(A, B, c, x0, H, h, Q_u):
    """Textbook backward Riccati recursion and forward rollout."""
    N, n_s = h.shape
    R = 2 * Q_u
    P, p = H[-1].copy(), h[-1].copy()
    Ks, ks = [None] * N, [None] * N
    for t in range(N - 1, -1, -1):
        Quu = R + B.T @ P @ B
        Qux = B.T @ P @ A
        qu = B.T @ (P @ c + p)
        Ks[t] = -np.linalg.solve(Quu, Qux)
        ks[t] = -np.linalg.solve(Quu, qu)
        if t > 0:
            Pn = H[t - 1] + A.T @ P @ A + Qux.T @ Ks[t]
            pn = h[t - 1] + A.T @ (P @ c + p) + Qux.T @ ks[t]
            P, p = 0.5 * (Pn + Pn.T), pn
    x = [x0]
    u = []
    for t in range(N):
        u.append(Ks[t] @ x[-1] + ks[t])
        x.append(A @ x[-1] + B @ u[-1] + c)
    return np.array(x), np.array(u)


def random_lq(rng, n_s=4, n_u=2, N=12):
    A = np.eye(n_s) + 0.1 * rng.normal(size=(n_s, n_s))
    B = 0.2 * rng.normal(size=(n_s, n_u))
    c = 0.1 * rng.normal(size=n_s)
    H = []
    for _ in range(N):
        M = rng.normal(size=(n_s, n_s))
        H.append(M @ M.T + 0.5 * np.eye(n_s))
    H = np.array(H)
    h = rng.normal(size=(N, n_s))
    Q = rng.normal(size=(n_u, n_u))
    return A, B, c, rng.normal(size=n_s), H, h, Q @ Q.T + 0.2 * np.eye(n_u)


def test_traj_qp_vs_dense_kkt_and_riccati():
    rng = np.random.default_rng(0)
    for n_s, n_u in [(4, 2), (12, 4)]:
        for _ in range(3):
            prob = random_lq(rng, n_s, n_u)
            x, u = oracle.traj_qp(*prob)
            xd, ud = dense_kkt_lq(*prob)
            xr, ur = riccati_lq(*prob)
            assert np.allclose(x, xd, atol=1e-9, rtol=1e-9)
            assert np.allclose(u, ud, atol=1e-9, rtol=1e-9)
            assert np.allclose(x, xr, atol=1e-8, rtol=1e-8)


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_obstacle_free_lq_follows_consistent_reference(name):
    """The straight reference is a trajectory of the linearised model and
    x_0 is on it, so the obstacle-free LQ solution is the reference, u = 0."""
    p = workloads.make(name)
    N, n_s = p["N"], p["n_s"]
    H = np.array([2 * p["Q_s"]] * N)
    h = np.array([-2 * p["Q_s"] @ p["x_ref"][0, t] for t in range(1, N + 1)])
    x, u = oracle.traj_qp(p["A_dyn"], p["B_dyn"], p["c_dyn"], p["x0"][0], H, h, p["Q_u"])
    assert np.allclose(x, p["x_ref"][0], atol=1e-9)
    assert np.allclose(u, 0.0, atol=1e-9)


def scale_certificate_state(P, p):
    st = P.init_state()
    return st


@pytest.mark.parametrize("name,seed", [("c1", 16), ("c2", 10), ("c3", 25)])
def test_T_R_at_scale_certificate(name, seed):
    """At the scale-LP certificate y0 = (lam*, mu*, max(alpha*-1, 0)),
    T = 1 + d'^T mu + gamma = max(0, 1 - alpha*) and R = 0 (Sec. III-B, IV-A)."""
    p = workloads.make(name, seed=seed)
    P = oracle.Problem(p)
    st = P.init_state()
    alpha = P.scale_all(st["x"])
    T, R, _ = P.mult_phase(st["x"], st["y"], np.zeros_like(st["zeta"]), np.zeros_like(st["xi"]))
    assert np.allclose(T, np.maximum(0.0, 1.0 - alpha), atol=1e-9)
    assert np.allclose(R, 0.0, atol=1e-9)


def fd_jacobians(P, p, x, y, h=1e-6):
    """Central differences of (T, R) of every pair w.r.t. each pose coordinate
    of its own x_t, through the oracle's multiplier update (zeta = xi = 0)."""
    qidx = list(p["pos_idx"]) + list(p["att_idx"])
    z0 = np.zeros(P.n_blocks * p["N"])
    x0 = np.zeros(P.n_blocks * p["N"] * p["dim"])
    J = []
    for c in qidx:
        xp, xm = x.copy(), x.copy()
        xp[:, 1:, c] += h
        xm[:, 1:, c] -= h
        Tp, Rp, _ = P.mult_phase(xp, y, z0, x0)
        Tm, Rm, _ = P.mult_phase(xm, y, z0, x0)
        J.append(((Tp - Tm) / (2 * h), (Rp - Rm) / (2 * h)))
    return qidx, J


@pytest.mark.parametrize("name,seed", [("c1", 16), ("c3", 25)])
def test_traj_phase_vs_fd_linearisation(name, seed):
    """The state update solves min F + sigma/2 sum ||r + J (q - q^k)||^2 with J
    the Jacobian of (T, R) in the pose coordinates at s^k (Sec. IV-B, SQP
    step). Rebuild that QP with finite-difference Jacobians and a dense KKT
    solve and compare with the oracle's state update."""
    p = workloads.make(name, seed=seed)
    P = oracle.Problem(p)
    st = P.init_state()
    for _ in range(3):   # move away from the initial point first
        y1 = P.pair_phase(st)
        x1, u1 = P.traj_phase(st, y1)
        z1, xi1, _ = P.mult_phase(x1, y1, st["zeta"], st["xi"])
        st.update(x=x1, u=u1, y=y1, zeta=z1, xi=xi1)
    y1 = P.pair_phase(st)
    x_orc, u_orc = P.traj_phase(st, y1)
    N, n_s, dim = p["N"], p["n_s"], p["dim"]
    nb = P.n_blocks
    T0, R0, _ = P.mult_phase(st["x"], y1, np.zeros(nb * N), np.zeros(nb * N * dim))
    r0 = T0 + st["zeta"]
    rR = (R0 + st["xi"]).reshape(nb, dim, N)
    qidx, J = fd_jacobians(P, p, st["x"], y1)
    nq = len(qidx)
    H = np.array([2 * p["Q_s"]] * N)
    h = np.array([-2 * p["Q_s"] @ p["x_ref"][0, t] for t in range(1, N + 1)])
    sig = p["sigma"]
    for b in range(nb):
        for t in range(N):
            Jm = np.zeros((dim + 1, n_s))
            for a in range(nq):
                JT, JR = J[a]
                Jm[0, qidx[a]] = JT[b * N + t]
                Jm[1:, qidx[a]] = JR.reshape(nb, dim, N)[b, :, t]
            r = np.r_[r0[b * N + t], rR[b, :, t]]
            xk = st["x"][0, t + 1]
            H[t] += sig * Jm.T @ Jm
            h[t] += sig * Jm.T @ (r - Jm @ xk)
    xd, ud = dense_kkt_lq(p["A_dyn"], p["B_dyn"], p["c_dyn"], p["x0"][0], H, h, p["Q_u"])
    scale = np.abs(xd).max()
    assert np.allclose(x_orc[0], xd, atol=1e-6 * scale)
    assert np.allclose(u_orc[0], ud, atol=1e-5 * max(1.0, np.abs(ud).max()))


def test_far_obstacles_fixed_point():
    """If every pair has alpha* >= 1 along s^0 the iteration is stationary from
    the first step: s^k = s^0, zeta = xi = 0, y^k = y^0."""
    p = workloads.make("c1", seed=3)
    P = oracle.Problem(p)
    st = P.init_state()
    assert P.scale_all(st["x"]).min() > 1.0
    ref = {k: v.copy() for k, v in st.items()}
    hist = P.run(st, 5)
    assert hist["iters"][0] == 1
    assert np.allclose(st["x"], ref["x"], atol=1e-12)
    assert np.allclose(st["y"], ref["y"], atol=1e-12)
    assert np.abs(st["zeta"]).max() < 1e-12 and np.abs(st["xi"]).max() < 1e-12


def test_no_obstacles_gives_lq_solution():
    p = workloads.make("c1", seed=16)
    p = workloads.with_obstacles(p, [[]])
    P = oracle.Problem(p)
    st = P.init_state()
    P.run(st, 3)
    assert np.allclose(st["x"][0], p["x_ref"][0], atol=1e-9)


def test_convergence_gives_certificate():
    """At convergence T ~ 0 and R ~ 0, so (lam, mu) certifies
    -d'^T mu = 1 + gamma >= 1 and the scale LP gives alpha* close to >= 1
    (Sec. III-B)."""
    p = workloads.make("c1", seed=16)
    P = oracle.Problem(p)
    st = P.init_state()
    assert P.scale_all(st["x"]).min() < 0.5
    hist = P.run(st, 200)
    k = hist["iters"][0]
    assert k < 200
    assert hist["r_pri"][k - 1, 0] <= p["eps_pri"] and hist["r_dual"][k - 1, 0] <= p["eps_dual"]
    # the stop test fired at the first iteration where both hold
    both = (hist["r_pri"][:k, 0] <= p["eps_pri"]) & (hist["r_dual"][:k, 0] <= p["eps_dual"])
    assert both[-1] and not both[:-1].any()
    assert P.scale_all(st["x"]).min() > 0.97


def test_scenarios_are_separable():
    """Batched scenarios give the same iterates as separate runs (Sec. IV-B,
    separability of the sub-problems)."""
    p = workloads.config_c4(n_scen=3, m_range=(4, 8))
    P = oracle.Problem(p)
    st = P.init_state()
    P.run(st, 6)
    for s in range(3):
        q = workloads.select_scenarios(p, [s])
        Q = oracle.Problem(q)
        sq = Q.init_state()
        Q.run(sq, 6)
        assert np.array_equal(sq["x"][0], st["x"][s])
