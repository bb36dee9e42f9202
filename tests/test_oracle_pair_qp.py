"""Pins of the oracle's dual-update sub-problem (Sec. IV-C, eq.
const_least_square, with the Jacobi-scaled proximal term of the build's
reading) against brute force over active sets, a library NLP solver on the
definitional objective, KKT conditions and LP duality."""
import itertools

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
import workloads


def make_pair(rng, dim, n_pts=8, spread=4.0):
    h = rng.uniform(0.5, 2.0, dim)
    A = np.concatenate([np.eye(dim), -np.eye(dim)])
    b = np.concatenate([h, h])
    pts = workloads.disc_points(rng, n_pts, 2.0, dim)
    C, d = workloads.hull_faces(pts)
    c = rng.uniform(-spread, spread, dim)
    d = d + C @ c
    # a random attitude: Cp = C R, dp = d - C pos with pos = 0
    th = rng.uniform(-np.pi, np.pi)
    R = np.eye(dim)
    R[0, 0], R[0, 1], R[1, 0], R[1, 1] = np.cos(th), -np.sin(th), np.sin(th), np.cos(th)
    return A, b, C @ R, d


def K_of(A, Cp, dp):
    """Rows of K in the paper's order (Sec. IV-C): (0, A), (d', C'), (1, 0)."""
    nr, no, dim = len(A), len(dp), A.shape[1]
    K = np.zeros((nr + no + 1, dim + 1))
    K[:nr, 1:] = A
    K[nr:nr + no, 0] = dp
    K[nr:nr + no, 1:] = Cp
    K[-1, 0] = 1.0
    return K


def objective(y, A, b, Cp, dp, zeta, xi, yhat, eps):
    K = K_of(A, Cp, dp)
    r = K.T @ y + np.r_[1.0 + zeta, xi]
    D = (K ** 2).sum(1)
    return 0.5 * r @ r + 0.5 * eps * np.sum(D * (y - yhat) ** 2)


def random_inputs(rng, A, b, Cp, dp):
    n = len(b) + len(dp) + 1
    yhat = np.abs(rng.normal(size=n)) * (rng.uniform(size=n) < 0.5)
    yhat[:len(b)] = 0.0
    yhat[int(rng.integers(len(b)))] = 1.0
    yhat[:len(b)] /= b @ yhat[:len(b)]
    zeta = rng.normal()
    xi = 0.3 * rng.normal(size=A.shape[1])
    return zeta, xi, yhat


@pytest.mark.parametrize("eps", [1e-1, 1e-3])
def test_pair_qp_bruteforce_active_sets(eps):
    """Enumerate every free set of the bound constraints (n <= 12), solve each
    equality-constrained QP and keep the KKT point; it must be unique and equal
    the oracle's solution."""
    rng = np.random.default_rng(int(eps * 1e4))
    for _ in range(6):
        A, b, Cp, dp = make_pair(rng, 2, n_pts=7)
        n = len(b) + len(dp) + 1
        if n > 12:
            continue
        zeta, xi, yhat = random_inputs(rng, A, b, Cp, dp)
        K = K_of(A, Cp, dp)
        D = (K ** 2).sum(1)
        G = K @ K.T + eps * np.diag(D)
        g = K @ np.r_[1 + zeta, xi] - eps * D * yhat
        kap = np.r_[b, np.zeros(n - len(b))]
        kkt_points = []
        for mask in range(1, 1 << n):
            F = [l for l in range(n) if mask >> l & 1]
            if not np.any(kap[F] > 0):
                continue
            m = len(F)
            M = np.zeros((m + 1, m + 1))
            M[:m, :m] = G[np.ix_(F, F)]
            M[:m, m] = -kap[F]
            M[m, :m] = kap[F]
            sol = np.linalg.solve(M, np.r_[-g[F], 1.0])
            y = np.zeros(n)
            y[F] = sol[:m]
            nu = sol[m]
            if np.any(y < -1e-12):
                continue
            w = G @ y + g - kap * nu
            if np.any(w < -1e-9):
                continue
            kkt_points.append(y)
        assert len(kkt_points) >= 1
        for y in kkt_points[1:]:
            assert np.allclose(y, kkt_points[0], atol=1e-9)
        y_orc, it = oracle.pair_qp(A, b, Cp, dp, zeta, xi, yhat, eps)
        assert it >= 0
        assert np.allclose(y_orc, kkt_points[0], atol=1e-9, rtol=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
def test_pair_qp_vs_library_solver(dim):
    """The oracle's y is feasible and no worse than SLSQP on the definitional
    objective; by strict convexity both are the same point."""
    rng = np.random.default_rng(40 + dim)
    for _ in range(8):
        A, b, Cp, dp = make_pair(rng, dim, n_pts=7)
        zeta, xi, yhat = random_inputs(rng, A, b, Cp, dp)
        eps = 0.1
        y, it = oracle.pair_qp(A, b, Cp, dp, zeta, xi, yhat, eps)
        assert it >= 0
        assert np.all(y >= 0) and b @ y[:len(b)] == pytest.approx(1.0, abs=1e-12)
        n = len(y)
        cons = [{"type": "eq", "fun": lambda z: b @ z[:len(b)] - 1.0,
                 "jac": lambda z: np.r_[b, np.zeros(n - len(b))]}]
        f = lambda z: objective(z, A, b, Cp, dp, zeta, xi, yhat, eps)
        res = minimize(f, yhat, method="SLSQP", bounds=[(0, None)] * n, constraints=cons,
                       options={"ftol": 1e-14, "maxiter": 500})
        assert f(y) <= res.fun + 1e-10
        assert np.allclose(y, res.x, atol=2e-5)


def test_pair_qp_kkt_residuals():
    """Stationarity, complementarity and feasibility (Sec. IV-C, eq.
    kkt_conditions adapted to the equality form) on 3D pairs."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        A, b, Cp, dp = make_pair(rng, 3, n_pts=10)
        zeta, xi, yhat = random_inputs(rng, A, b, Cp, dp)
        eps = 0.1
        y, it = oracle.pair_qp(A, b, Cp, dp, zeta, xi, yhat, eps)
        assert it >= 0
        K = K_of(A, Cp, dp)
        D = (K ** 2).sum(1)
        grad = K @ (K.T @ y + np.r_[1 + zeta, xi]) + eps * D * (y - yhat)
        kap = np.r_[b, np.zeros(len(y) - len(b))]
        F = y > 0
        # nu from the free lambda rows, then bound multipliers w = grad - kap nu
        nu = np.linalg.lstsq(kap[F][:, None], grad[F], rcond=None)[0][0]
        w = grad - kap * nu
        scale = max(1.0, np.abs(grad).max())
        assert np.allclose(w[F], 0.0, atol=1e-9 * scale)
        assert np.all(w[~F] >= -1e-9 * scale)
        assert b @ y[:len(b)] == pytest.approx(1.0, abs=1e-12)


def test_zero_multiplier_value_vs_scale():
    """With zeta = xi = 0 and a vanishing proximal weight the optimal value is
    0 exactly when a collision-free certificate exists, i.e. alpha* >= 1
    (Sec. III-B strong duality)."""
    rng = np.random.default_rng(9)
    seen = {True: 0, False: 0}
    for _ in range(120):
        A, b, Cp, dp = make_pair(rng, 2, n_pts=9, spread=5.0)
        alpha = oracle.scale_lp(A, b, Cp, dp)[0]
        if abs(alpha - 1.0) < 0.05:
            continue
        n = len(b) + len(dp) + 1
        yhat = np.zeros(n)
        y, it = oracle.pair_qp(A, b, Cp, dp, 0.0, np.zeros(2), yhat, 1e-10)
        assert it >= 0
        val = objective(y, A, b, Cp, dp, 0.0, np.zeros(2), yhat, 0.0)
        free = alpha >= 1.0
        assert (val < 1e-8) == free
        seen[free] += 1
    assert seen[True] > 10 and seen[False] > 10


def test_certificate_is_fixed_point():
    """At the LP certificate y = (lam*, mu*, alpha* - 1) with alpha* >= 1 and
    zeta = xi = 0 the residual K^T y + bhat vanishes, so the proximal
    sub-problem returns its centre exactly."""
    rng = np.random.default_rng(11)
    done = 0
    for _ in range(60):
        A, b, Cp, dp = make_pair(rng, 2, n_pts=9, spread=6.0)
        alpha, x, lam, mu, gap, st = oracle.scale_lp(A, b, Cp, dp)
        if alpha < 1.0:
            continue
        yhat = np.r_[lam, mu, alpha - 1.0]
        y, it = oracle.pair_qp(A, b, Cp, dp, 0.0, np.zeros(2), yhat, 0.1)
        assert np.allclose(y, yhat, atol=1e-10)
        done += 1
    assert done > 10


def test_row_rescaling_invariance():
    """Scaling an obstacle face (c_l, d_l) by s > 0 maps y_l -> y_l / s and
    leaves every other entry unchanged (Jacobi-scaled proximal term)."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        A, b, Cp, dp = make_pair(rng, 2, n_pts=8)
        zeta, xi, yhat = random_inputs(rng, A, b, Cp, dp)
        y0, _ = oracle.pair_qp(A, b, Cp, dp, zeta, xi, yhat, 0.1)
        s = rng.uniform(0.2, 5.0, len(dp))
        yh1 = yhat.copy()
        yh1[len(b):len(b) + len(dp)] /= s
        y1, _ = oracle.pair_qp(A, b, Cp * s[:, None], dp * s, zeta, xi, yh1, 0.1)
        y1[len(b):len(b) + len(dp)] *= s
        assert np.allclose(y1, y0, atol=1e-9)


@pytest.mark.parametrize("dim,eps", [(2, 1e-1), (3, 1e-1), (2, 1e-3), (3, 1e-3)])
def test_lemke_route_equals_active_set(dim, eps):
    """The paper's route (Sec. IV-C: the equality eliminated, eq.
    const_least_square_ineq; its KKT conditions as the LCP of eq.
    linear_complementarity_problem; Lemke's method) and the primal
    active-set method give the same unique minimiser of the proximal QP."""
    rng = np.random.default_rng(31 + dim)
    worst = 0.0
    for _ in range(40):
        A, b, Cp, dp = make_pair(rng, dim, n_pts=9 if dim == 3 else 8)
        zeta, xi, yhat = random_inputs(rng, A, b, Cp, dp)
        y1, it = oracle.pair_qp(A, b, Cp, dp, zeta, xi, yhat, eps)
        y2, st = oracle.pair_qp_lemke(A, b, Cp, dp, zeta, xi, yhat, eps)
        assert it >= 0 and st == 0
        worst = max(worst, np.abs(y1 - y2).max() / max(1.0, np.abs(y1).max()))
    assert worst < 1e-8


def test_lemke_route_without_proximal_term_is_optimal():
    """eps = 0, the paper's QP as printed (Sec. IV-C eq. const_least_square):
    the minimiser is not unique (the Hessian K K^T has rank <= dim + 1), so
    the check is the KKT system of that QP, which certifies optimality of a
    convex QP: y >= 0, kappa^T y = 1, K (K^T y + b) - nu kappa = w >= 0,
    w^T y = 0; and the optimal value 0 exactly when alpha* >= 1 for zero
    multipliers (LP duality, Sec. III-B)."""
    rng = np.random.default_rng(5)
    for dim in (2, 3):
        for trial in range(30):
            A, b, Cp, dp = make_pair(rng, dim, n_pts=8)
            zeta, xi = (0.0, np.zeros(dim)) if trial % 2 == 0 else (rng.normal(), 0.3 * rng.normal(size=dim))
            yhat = np.zeros(len(b) + len(dp) + 1)
            y, st = oracle.pair_qp_lemke(A, b, Cp, dp, zeta, xi, yhat, 0.0)
            assert st == 0
            K = K_of(A, Cp, dp)
            kap = np.r_[b, np.zeros(len(dp) + 1)]
            r = K.T @ y + np.r_[1.0 + zeta, xi]
            g = K @ r
            free = y > 1e-9 * max(1.0, y.max())
            # nu from the free rows with kappa > 0 (least squares over them)
            fk = free & (kap > 0)
            nu = (g[fk] @ kap[fk]) / (kap[fk] @ kap[fk]) if fk.any() else 0.0
            w = g - nu * kap
            scale = 1.0 + np.abs(K).sum() * (1.0 + y.max())
            assert y.min() >= -1e-12 and abs(kap @ y - 1.0) < 1e-10
            assert np.abs(w[free]).max() < 1e-8 * scale
            assert w[~free].min() > -1e-8 * scale
            if trial % 2 == 0:
                alpha = oracle.scale_lp(A, b, Cp, dp)[0]
                val = 0.5 * r @ r
                if alpha > 1.0 + 1e-6:
                    assert val < 1e-12
                elif alpha < 1.0 - 1e-6:
                    assert val > 1e-12
