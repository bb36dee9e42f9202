"""Pins of the oracle's bounded trajectory QP (Sec. IV-A eq. MPC_opt_origin,
its state and control rows; the indicator IC_0 of Sec. IV-B eq.
ADMM_Lagrangian in the state update of eq. ADMM_state_updates):

    min sum_{t=1..N} 1/2 x_t^T H_t x_t + h_t^T x_t + sum_{t=0..N-1} u_t^T Q_u u_t
    s.t. x_{t+1} = A x_t + B u_t + c, s_lo <= x_t <= s_hi, u_lo <= u_t <= u_hi.

The QP is strictly convex, so its minimiser is unique and fixed by the KKT
conditions. Checked here without the oracle's condensing or its active-set
steps: brute force over every active set of the bounds in the stacked
variables (x_1..x_N, u_0..u_{N-1}) on small horizons, the KKT conditions at
larger sizes, SciPy's bounded least squares for input-only bounds, and the
plain LQ solution when no bound is active."""
import itertools

import numpy as np
import pytest

import oracle
import workloads


def random_lq(rng, n_s, n_u, N):
    A = np.eye(n_s) + 0.2 * rng.standard_normal((n_s, n_s))
    B = rng.standard_normal((n_s, n_u))
    c = 0.1 * rng.standard_normal(n_s)
    x0 = rng.standard_normal(n_s)
    H = np.zeros((N, n_s, n_s))
    for t in range(N):
        R = rng.standard_normal((n_s, n_s))
        H[t] = R @ R.T / n_s + 0.5 * np.eye(n_s)
    h = rng.standard_normal((N, n_s))
    R = rng.standard_normal((n_u, n_u))
    Q_u = R @ R.T / n_u + 0.3 * np.eye(n_u)
    return A, B, c, x0, H, h, Q_u


def stacked(A, B, c, x0, H, h, Q_u):
    """Objective 1/2 z^T P z + q^T z and dynamics E z = f in the stacked
    variables z = (x_1..x_N, u_0..u_{N-1})."""
    N, n_s = h.shape
    n_u = B.shape[1]
    nz = N * (n_s + n_u)
    xi = lambda t: slice((t - 1) * n_s, t * n_s)            # x_t, t = 1..N
    ui = lambda t: slice(N * n_s + t * n_u, N * n_s + (t + 1) * n_u)
    P = np.zeros((nz, nz))
    q = np.zeros(nz)
    for t in range(1, N + 1):
        P[xi(t), xi(t)] = H[t - 1]
        q[xi(t)] = h[t - 1]
    for t in range(N):
        P[ui(t), ui(t)] = 2.0 * Q_u
    E = np.zeros((N * n_s, nz))
    f = np.zeros(N * n_s)
    for t in range(N):
        r = slice(t * n_s, (t + 1) * n_s)
        E[r, xi(t + 1)] = np.eye(n_s)
        E[r, ui(t)] = -B
        if t == 0:
            f[r] = A @ x0 + c
        else:
            E[r, xi(t)] = -A
            f[r] = c
    return P, q, E, f


def bound_vectors(N, n_s, n_u, s_lo, s_hi, u_lo, u_hi):
    inf = np.full
    lo = np.concatenate([np.tile(s_lo if s_lo is not None else inf(n_s, -np.inf), N),
                         np.tile(u_lo if u_lo is not None else inf(n_u, -np.inf), N)])
    hi = np.concatenate([np.tile(s_hi if s_hi is not None else inf(n_s, np.inf), N),
                         np.tile(u_hi if u_hi is not None else inf(n_u, np.inf), N)])
    return lo, hi


def stack_solution(x, u):
    return np.concatenate([x[1:].ravel(), u.ravel()])


def brute_force(P, q, E, f, lo, hi, max_active):
    """Every set of at most max_active bounds held with equality: the
    equality-constrained QP's solution, kept if it is feasible and every bound
    multiplier has the right sign. The strictly convex QP has one such point."""
    nz = len(q)
    cands = [(v, -1) for v in range(nz) if np.isfinite(lo[v])] + [(v, 1) for v in range(nz) if np.isfinite(hi[v])]
    found = []
    for k in range(max_active + 1):
        for S in itertools.combinations(cands, k):
            vars_ = [v for v, _ in S]
            if len(set(vars_)) < len(vars_):
                continue
            m = E.shape[0]
            K = np.zeros((nz + m + k, nz + m + k))
            K[:nz, :nz] = P
            K[:nz, nz:nz + m] = E.T
            K[nz:nz + m, :nz] = E
            rhs = np.concatenate([-q, f, np.zeros(k)])
            for a, (v, side) in enumerate(S):
                K[v, nz + m + a] = 1.0
                K[nz + m + a, v] = 1.0
                rhs[nz + m + a] = hi[v] if side > 0 else lo[v]
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            z = sol[:nz]
            mu = sol[nz + m:]
            if np.any(z < lo - 1e-9) or np.any(z > hi + 1e-9):
                continue
            # P z + q + E^T lam + sum mu_a e_v = 0: an upper bound needs mu >= 0, a lower one mu <= 0
            if all(mu[a] * side >= -1e-9 for a, (_, side) in enumerate(S)):
                found.append(z)
    return found


@pytest.mark.parametrize("seed", range(6))
def test_bounded_qp_vs_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n_s, n_u, N = 2, 1, 3
    while True:
        A, B, c, x0, H, h, Q_u = random_lq(rng, n_s, n_u, N)
        x_f, u_f = oracle.traj_qp(A, B, c, x0, H, h, Q_u)
        # bounds that cut the unconstrained solution: inputs to 60% of its
        # largest magnitude, the first state's upper bound below its maximum
        a = 0.6 * np.abs(u_f).max()
        u_lo, u_hi = np.array([-a]), np.array([a])
        s_hi = np.array([x_f[1:, 0].max() - 0.3 * np.ptp(x_f[1:, 0]), np.inf])
        s_lo = np.array([-np.inf, x_f[1:, 1].min() + 0.2 * np.ptp(x_f[1:, 1])])
        P, q, E, f = stacked(A, B, c, x0, H, h, Q_u)
        lo, hi = bound_vectors(N, n_s, n_u, s_lo, s_hi, u_lo, u_hi)
        found = brute_force(P, q, E, f, lo, hi, N * n_u)
        if found:
            break
    assert len(found) == 1 or max(np.abs(z - found[0]).max() for z in found) < 1e-9
    x, u, na = oracle.traj_qp_bounded(A, B, c, x0, H, h, Q_u, s_lo, s_hi, u_lo, u_hi)
    z = stack_solution(x, u)
    assert np.abs(z - found[0]).max() <= 1e-9 * (1 + np.abs(found[0]).max())
    assert na >= 1
    assert np.allclose(x[0], x0)


def kkt_residuals(P, q, E, f, lo, hi, z, tol):
    """Stationarity residual with the multipliers fitted by least squares on
    the bounds held at z (within tol), the largest wrong-signed bound
    multiplier and the largest bound violation."""
    nz = len(q)
    act = [(v, 1.0) for v in range(nz) if np.isfinite(hi[v]) and z[v] >= hi[v] - tol]
    act += [(v, -1.0) for v in range(nz) if np.isfinite(lo[v]) and z[v] <= lo[v] + tol]
    G = np.hstack([E.T] + [np.eye(nz)[:, [v]] for v, _ in act]) if act else E.T
    g = -(P @ z + q)
    mult, *_ = np.linalg.lstsq(G, g, rcond=None)
    stat = np.abs(G @ mult - g).max()
    mu = mult[E.shape[0]:]
    wrong = max([0.0] + [-(mu[a] * side) for a, (_, side) in enumerate(act)])
    viol = max(0.0, np.max(lo - z), np.max(z - hi))
    return stat, wrong, viol, len(act), np.abs(E @ z - f).max()


def feasible(E, f, lo, hi):
    """Whether any point meets the dynamics and the bounds (HiGHS LP)."""
    from scipy.optimize import linprog
    bnd = [(a if np.isfinite(a) else None, b if np.isfinite(b) else None) for a, b in zip(lo, hi)]
    return linprog(np.zeros(len(lo)), A_eq=E, b_eq=f, bounds=bnd, method="highs").status == 0


@pytest.mark.parametrize("n_s,n_u,N,seed", [(4, 2, 20, 0), (4, 2, 30, 1), (12, 4, 12, 2), (3, 2, 15, 5)])
def test_bounded_qp_kkt(n_s, n_u, N, seed):
    rng = np.random.default_rng(200 + seed)
    A, B, c, x0, H, h, Q_u = random_lq(rng, n_s, n_u, N)
    A = 0.95 * A / max(1.0, np.abs(np.linalg.eigvals(A)).max())
    x_f, u_f = oracle.traj_qp(A, B, c, x0, H, h, Q_u)
    P, q, E, f = stacked(A, B, c, x0, H, h, Q_u)
    # cut the unconstrained solution by bounds on the inputs and two states,
    # less and less until a feasible point exists
    for cut in (0.3, 0.2, 0.1, 0.05):
        u_hi = (1 - cut) * 0.7 * np.abs(u_f).max(axis=0)
        u_lo = -(1 - cut) * np.abs(u_f).max(axis=0)
        # (above what the first two steps reach: x_1 and x_2 barely move)
        s_hi = np.maximum(x_f[3:].max(axis=0) - cut * np.ptp(x_f[1:], axis=0), x_f[1:3].max(axis=0) + 1e-3)
        s_hi[2:] = np.inf
        lo, hi = bound_vectors(N, n_s, n_u, None, s_hi, u_lo, u_hi)
        if feasible(E, f, lo, hi):
            break
    x, u, na = oracle.traj_qp_bounded(A, B, c, x0, H, h, Q_u, None, s_hi, u_lo, u_hi)
    z = stack_solution(x, u)
    scale = 1 + np.abs(P @ z).max() + np.abs(q).max()
    stat, wrong, viol, n_act, dyn = kkt_residuals(P, q, E, f, lo, hi, z, 1e-9 * (1 + np.abs(z).max()))
    assert n_act == na and na >= 2
    assert stat <= 1e-9 * scale
    assert wrong <= 1e-9 * scale
    assert viol <= 1e-9 * (1 + np.abs(z).max())
    assert dyn <= 1e-10 * (1 + np.abs(z).max())


def unit_response(A, B, N, n_s, n_u):
    """dx_t/du by simulating each unit input separately (t = 1..N)."""
    S = np.zeros((N * n_s, N * n_u))
    for col in range(N * n_u):
        uu = np.zeros(N * n_u)
        uu[col] = 1.0
        xx = np.zeros(n_s)
        for t in range(N):
            xx = A @ xx + B @ uu[t * n_u:(t + 1) * n_u]
            S[t * n_s:(t + 1) * n_s, col] = xx
    return S


@pytest.mark.parametrize("seed", range(3))
def test_input_bounds_vs_bounded_least_squares(seed):
    from scipy.optimize import lsq_linear
    rng = np.random.default_rng(300 + seed)
    n_s, n_u, N = 4, 2, 25
    A, B, c, x0, H, h, Q_u = random_lq(rng, n_s, n_u, N)
    A = 0.95 * A / max(1.0, np.abs(np.linalg.eigvals(A)).max())
    x_f, u_f = oracle.traj_qp(A, B, c, x0, H, h, Q_u)
    u_hi = 0.4 * np.abs(u_f).max(axis=0)
    u_lo = -0.4 * np.abs(u_f).max(axis=0)
    x, u, na = oracle.traj_qp_bounded(A, B, c, x0, H, h, Q_u, None, None, u_lo, u_hi)
    # free response and the unit responses, then the least-squares form of
    # 1/2 u^T G u + g^T u with G = L L^T: || L^T u + L^{-1} g ||^2
    zf = np.zeros(N * n_s)
    xx = x0.copy()
    for t in range(N):
        xx = A @ xx + c
        zf[t * n_s:(t + 1) * n_s] = xx
    S = unit_response(A, B, N, n_s, n_u)
    Hb = np.zeros((N * n_s, N * n_s))
    for t in range(N):
        Hb[t * n_s:(t + 1) * n_s, t * n_s:(t + 1) * n_s] = H[t]
    G = S.T @ Hb @ S + np.kron(np.eye(N), 2.0 * Q_u)
    g = S.T @ (Hb @ zf + h.ravel())
    L = np.linalg.cholesky(G)
    res = lsq_linear(L.T, -np.linalg.solve(L, g), bounds=(np.tile(u_lo, N), np.tile(u_hi, N)),
                     method="bvls", tol=1e-13)
    assert np.abs(u.ravel() - res.x).max() <= 1e-8 * (1 + np.abs(res.x).max())
    assert na >= 2


def test_inactive_bounds_give_the_lq_solution():
    rng = np.random.default_rng(400)
    A, B, c, x0, H, h, Q_u = random_lq(rng, 4, 2, 20)
    A = 0.95 * A / max(1.0, np.abs(np.linalg.eigvals(A)).max())
    x_f, u_f = oracle.traj_qp(A, B, c, x0, H, h, Q_u)
    big = 10 * (1 + max(np.abs(x_f).max(), np.abs(u_f).max()))
    x, u, na = oracle.traj_qp_bounded(A, B, c, x0, H, h, Q_u, np.full(4, -big), np.full(4, big),
                                      np.full(2, -big), np.full(2, big))
    assert na == 0
    assert np.abs(x - x_f).max() <= 1e-10 * (1 + np.abs(x_f).max())
    assert np.abs(u - u_f).max() <= 1e-10 * (1 + np.abs(u_f).max())


def test_infeasible_bounds_are_reported():
    """A state bound that x_1 cannot meet from x_0 (x_1 = x_0 + u_0 with
    |u_0| <= 1 and x_1 >= x_0 + 5)."""
    A, B, c = np.eye(1), np.ones((1, 1)), np.zeros(1)
    x0 = np.zeros(1)
    H = np.ones((2, 1, 1))
    h = np.zeros((2, 1))
    with pytest.raises(RuntimeError):
        oracle.traj_qp_bounded(A, B, c, x0, H, h, np.eye(1), np.array([5.0]), None, np.array([-1.0]),
                               np.array([1.0]))



@pytest.mark.parametrize("seed", range(4))
def test_infeasibility_agrees_with_linear_programming(seed):
    """Tight random bounds: the oracle reports infeasibility exactly when an
    LP finds no point that meets the dynamics and the bounds."""
    rng = np.random.default_rng(500 + seed)
    n_s, n_u, N = 3, 2, 10
    A, B, c, x0, H, h, Q_u = random_lq(rng, n_s, n_u, N)
    A = 0.95 * A / max(1.0, np.abs(np.linalg.eigvals(A)).max())
    x_f, u_f = oracle.traj_qp(A, B, c, x0, H, h, Q_u)
    u_hi = rng.uniform(0.1, 0.6) * np.abs(u_f).max(axis=0)
    s_hi = x_f[1:].max(axis=0) - rng.uniform(0.1, 0.5) * np.ptp(x_f[1:], axis=0)
    P, q, E, f = stacked(A, B, c, x0, H, h, Q_u)
    lo, hi = bound_vectors(N, n_s, n_u, None, s_hi, -u_hi, u_hi)
    ok = feasible(E, f, lo, hi)
    if ok:
        oracle.traj_qp_bounded(A, B, c, x0, H, h, Q_u, None, s_hi, -u_hi, u_hi)
    else:
        with pytest.raises(RuntimeError):
            oracle.traj_qp_bounded(A, B, c, x0, H, h, Q_u, None, s_hi, -u_hi, u_hi)
