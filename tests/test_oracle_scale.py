"""Pins of the oracle's scale LP (Sec. III-A eq. scale_opt; Sec. III-B eq.
scale_opt_dual) against closed forms, brute force, a library LP solver,
strong duality and the collision semantics of alpha*."""
import itertools
import os

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def box_A(h):
    d = len(h)
    return np.concatenate([np.eye(d), -np.eye(d)]), np.concatenate([h, h])


def load_box_golden():
    rows = []
    with open(os.path.join(HERE, "golden", "box_scale.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            dim, h, lo, hi, a = [s.strip() for s in line.split("|")]
            rows.append((int(dim), np.array(h.split(), float), np.array(lo.split(), float),
                         np.array(hi.split(), float), float(a)))
    return rows


@pytest.mark.parametrize("case", load_box_golden())
def test_box_closed_form_golden(case):
    dim, h, lo, hi, expect = case
    A, b = box_A(h)
    C, d = box_A(np.ones(dim))
    d = np.concatenate([hi, -lo])
    alpha, x, lam, mu, gap, st = oracle.scale_lp(A, b, C, d)
    assert st == 0
    assert alpha == pytest.approx(expect, rel=1e-12, abs=1e-12)


def test_box_closed_form_random():
    rng = np.random.default_rng(1)
    for _ in range(200):
        dim = int(rng.integers(2, 4))
        h = rng.uniform(0.1, 3.0, dim)
        c = rng.uniform(-10, 10, dim)
        w = rng.uniform(0.1, 4.0, dim)
        lo, hi = c - w, c + w
        expect = max(0.0, np.max(np.maximum(lo / h, -hi / h)))
        A, b = box_A(h)
        C = np.concatenate([np.eye(dim), -np.eye(dim)])
        d = np.concatenate([hi, -lo])
        alpha, x, lam, mu, gap, st = oracle.scale_lp(A, b, C, d)
        assert st == 0
        assert alpha == pytest.approx(expect, rel=1e-10, abs=1e-10)


def vertex_enum_alpha(A, b, C, d):
    """Brute force over all (dim+1)-subsets of the constraints of
    min alpha s.t. A x - alpha b <= 0, C x <= d in variables (alpha, x)."""
    dim = A.shape[1]
    G = np.concatenate([np.concatenate([-b[:, None], A], 1),
                        np.concatenate([np.zeros((len(d), 1)), C], 1)])
    h = np.concatenate([np.zeros(len(b)), d])
    best = np.inf
    for S in itertools.combinations(range(len(h)), dim + 1):
        M = G[list(S)]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        z = np.linalg.solve(M, h[list(S)])
        if np.all(G @ z <= h + 1e-9):
            best = min(best, z[0])
    return best


def random_polytope(rng, dim, n_pts, r, centre):
    pts = workloads.disc_points(rng, n_pts, r, dim)
    C, d = workloads.hull_faces(pts)
    return C, d + C @ centre


def random_robot(rng, dim):
    h = rng.uniform(0.3, 2.0, dim)
    A, b = box_A(h)
    # rotate the part so its normals are not axis aligned
    th = rng.uniform(0, 2 * np.pi)
    R = np.eye(dim)
    R[0, 0], R[0, 1], R[1, 0], R[1, 1] = np.cos(th), -np.sin(th), np.sin(th), np.cos(th)
    return A @ R.T, b


@pytest.mark.parametrize("dim", [2, 3])
def test_vertex_enumeration_and_linprog(dim):
    rng = np.random.default_rng(10 + dim)
    for _ in range(40):
        A, b = random_robot(rng, dim)
        C, d = random_polytope(rng, dim, 8 if dim == 2 else 7, 1.5, rng.uniform(-4, 4, dim))
        alpha, x, lam, mu, gap, st = oracle.scale_lp(A, b, C, d)
        assert st == 0
        a_bf = vertex_enum_alpha(A, b, C, d)
        assert alpha == pytest.approx(a_bf, rel=1e-9, abs=1e-9)
        # library LP (HiGHS) on the primal in variables (alpha, x)
        G = np.concatenate([np.concatenate([-b[:, None], A], 1),
                            np.concatenate([np.zeros((len(d), 1)), C], 1)])
        hh = np.concatenate([np.zeros(len(b)), d])
        res = linprog(np.r_[1.0, np.zeros(dim)], A_ub=G, b_ub=hh,
                      bounds=[(None, None)] * (dim + 1), method="highs")
        assert res.status == 0
        assert alpha == pytest.approx(res.fun, rel=1e-8, abs=1e-8)


@pytest.mark.parametrize("dim", [2, 3])
def test_strong_duality_and_certificate(dim):
    """alpha* = -d^T mu* (Sec. III-B), dual feasibility of (lam*, mu*) and
    primal feasibility of (alpha*, x*)."""
    rng = np.random.default_rng(20 + dim)
    for _ in range(100):
        A, b = random_robot(rng, dim)
        C, d = random_polytope(rng, dim, 10, 2.0, rng.uniform(-6, 6, dim))
        alpha, x, lam, mu, gap, st = oracle.scale_lp(A, b, C, d)
        assert st == 0
        assert abs(gap) < 1e-9 * max(1.0, alpha)
        assert alpha == pytest.approx(-d @ mu, rel=1e-9, abs=1e-9)
        assert np.all(lam >= -1e-12) and np.all(mu >= -1e-12)
        assert b @ lam == pytest.approx(1.0, abs=1e-10)
        assert np.allclose(A.T @ lam + C.T @ mu, 0.0, atol=1e-9)
        assert np.all(A @ x <= alpha * b + 1e-9)
        assert np.all(C @ x <= d + 1e-9)


def test_invariances():
    rng = np.random.default_rng(5)
    for _ in range(50):
        A, b = random_robot(rng, 2)
        C, d = random_polytope(rng, 2, 12, 2.0, rng.uniform(-6, 6, 2))
        a0 = oracle.scale_lp(A, b, C, d)[0]
        c = rng.uniform(0.3, 3.0)
        # obstacle scaled about the robot centre: alpha scales by c
        assert oracle.scale_lp(A, b, C, c * d)[0] == pytest.approx(c * a0, rel=1e-9, abs=1e-9)
        # robot scaled by c: alpha scales by 1/c
        assert oracle.scale_lp(A, c * b, C, d)[0] == pytest.approx(a0 / c, rel=1e-9, abs=1e-9)
        # positive row rescaling of any face leaves alpha unchanged
        s_o = rng.uniform(0.2, 5.0, len(d))
        s_r = rng.uniform(0.2, 5.0, len(b))
        a1 = oracle.scale_lp(A * s_r[:, None], b * s_r, C * s_o[:, None], d * s_o)[0]
        assert a1 == pytest.approx(a0, rel=1e-9, abs=1e-9)


def polygon_vertices(C, d):
    """Vertices of a bounded 2D H-polytope by pairwise face intersection."""
    V = []
    for i, j in itertools.combinations(range(len(d)), 2):
        M = C[[i, j]]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        v = np.linalg.solve(M, d[[i, j]])
        if np.all(C @ v <= d + 1e-9):
            V.append(v)
    return np.array(V)


def sat_disjoint(C1, d1, C2, d2):
    """Separating-axis test for two convex polygons (edge normals as axes)."""
    V1, V2 = polygon_vertices(C1, d1), polygon_vertices(C2, d2)
    for n in np.concatenate([C1, C2]):
        if (V1 @ n).max() < (V2 @ n).min() - 1e-9 or (V2 @ n).max() < (V1 @ n).min() - 1e-9:
            return True
    return False


def test_alpha_vs_separating_axis():
    """alpha* > 1 iff the robot part and the obstacle are disjoint
    (Sec. III-A), checked against a textbook separating-axis test in the
    world frame with the part posed by R(theta), pos."""
    rng = np.random.default_rng(7)
    seen = {True: 0, False: 0}
    for _ in range(300):
        h = rng.uniform(0.5, 2.5, 2)
        A, b = box_A(h)
        th = rng.uniform(-np.pi, np.pi)
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        pos = rng.uniform(-3, 3, 2)
        C, d = random_polytope(rng, 2, 12, 2.0, rng.uniform(-3, 3, 2))
        # obstacle in the part frame: Cp = C R, dp = d - C pos
        alpha = oracle.scale_lp(A, b, C @ R, d - C @ pos)[0]
        if abs(alpha - 1.0) < 1e-6:
            continue
        # robot in the world frame: {y : A R^T (y - pos) <= b}
        Aw, bw = A @ R.T, b + A @ R.T @ pos
        disjoint = sat_disjoint(Aw, bw, C, d)
        assert disjoint == (alpha > 1.0)
        seen[disjoint] += 1
    assert seen[True] > 20 and seen[False] > 20
