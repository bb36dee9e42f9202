"""Pins of the oracle's reverse pass through the unrolled iteration (the
gradient of the tracking cost after K iterations with respect to the obstacle
face offsets d and the initial state x0, initial duals held fixed).

The pins are FP64 central differences (h = 1e-6) of the oracle's own forward
map, at an initial dual that is not an exact fixed point: at the scale-LP
certificate every inactive obstacle row of a far pair has a zero multiplier,
the pair QP's solution map has a kink there, and central differences average
the two one-sided derivatives. The sub-steps are pinned separately: the pair
QP's KKT-transpose VJP and the trajectory QP's VJP against differences of the
oracle's own sub-solvers."""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_pair_qp import make_pair, random_inputs


def fd(f, x0, h=1e-6):
    g = np.zeros(x0.size)
    for i in range(x0.size):
        e = np.zeros(x0.size)
        e.flat[i] = h
        g[i] = (f(x0 + e) - f(x0 - e)) / (2 * h)
    return g


def test_pair_qp_vjp_vs_differences():
    rng = np.random.default_rng(5)
    for _ in range(6):
        A, b, Cp, dp = make_pair(rng, 2, n_pts=7)
        zeta, xi, yhat = random_inputs(rng, A, b, Cp, dp)
        ybar = rng.normal(size=len(b) + len(dp) + 1)
        dpb, Cpb, zb, xib, yhb = oracle.pair_qp_vjp(A, b, Cp, dp, zeta, xi, yhat, 0.1, ybar)
        f = lambda **kw: ybar @ oracle.pair_qp(kw.get("A", A), b, kw.get("Cp", Cp), kw.get("dp", dp),
                                             kw.get("z", zeta), kw.get("xi", xi), kw.get("yh", yhat), 0.1)[0]
        assert np.allclose(dpb, fd(lambda v: f(dp=v), dp), rtol=1e-6, atol=1e-8)
        assert np.allclose(Cpb.ravel(), fd(lambda v: f(Cp=v.reshape(Cp.shape)), Cp.ravel()), rtol=1e-6, atol=1e-8)
        assert np.allclose(yhb, fd(lambda v: f(yh=v), yhat), rtol=1e-6, atol=1e-8)
        assert zb == pytest.approx(fd(lambda v: f(z=v[0]), np.array([zeta]))[0], rel=1e-6, abs=1e-8)
        assert np.allclose(xib, fd(lambda v: f(xi=v), xi), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_trajectory_vjp_vs_differences(name):
    p = workloads.make(name)
    P = oracle.Problem(p)
    st = P.init_state()
    P.run(st, 3)
    y1 = P.pair_phase(st)
    rng = np.random.default_rng(0)
    xbar = rng.normal(size=st["x"].shape)
    xbar[:, 0] = 0
    ubar = rng.normal(size=st["u"].shape)
    v = P.traj_vjp(st, y1, xbar, ubar)

    def f(st_=st, y_=y1, pp=P):
        x, u = pp.traj_phase(st_, y_)
        return (xbar * x).sum() + (ubar * u).sum()

    def fd_key(key, i, h=1e-6):
        a = dict(st)
        arr = st[key].copy(); arr.flat[i] += h; a[key] = arr; fp = f(st_=a)
        arr = st[key].copy(); arr.flat[i] -= h; a[key] = arr; fm = f(st_=a)
        return (fp - fm) / (2 * h)

    # central differences of f = xbar.x + ubar.u carry a rounding floor of
    # about |f| 1e-16 / h, amplified by the condition of the LQ solve
    f0 = abs(f())
    floor = 1e-8 * max(1.0, f0)

    def close(a, b):
        return abs(a - b) <= 1e-5 * abs(b) + floor

    for key in ("zeta", "xi"):
        for i in np.argsort(-np.abs(v[key]))[:4]:
            assert close(v[key][i], fd_key(key, i))
    for i in np.argsort(-np.abs(v["y"]))[:6]:
        a = y1.copy(); a[i] += 1e-6; fp = f(y_=a); a = y1.copy(); a[i] -= 1e-6; fm = f(y_=a)
        assert close(v["y"][i], (fp - fm) / 2e-6)
    for i in np.argsort(-np.abs(v["x"].ravel()))[:6]:
        assert close(v["x"].flat[i], fd_key("x", i))
    for i in np.argsort(-np.abs(v["d"]))[:4]:
        def g(h):
            q = dict(p); arr = p["obs_d"].copy(); arr[i] += h; q["obs_d"] = arr
            return f(pp=oracle.Problem(q))
        assert close(v["d"][i], (g(1e-6) - g(-1e-6)) / 2e-6)


@pytest.mark.parametrize("name,K,h,floor", [("c1", 1, 1e-6, 1e-9), ("c1", 10, 1e-6, 1e-9), ("c3", 4, 1e-6, 3e-7)])
def test_unrolled_gradient_vs_central_differences(name, K, h, floor):
    """h = 1e-6 throughout. The differences carry an absolute rounding floor:
    about 1e-9 for the planar model and about 3e-7 for the 12-state quadrotor,
    whose LQ solves are worse conditioned (measured by comparing h = 1e-5,
    1e-6 and 1e-7; larger steps add curvature error on the attitude)."""
    p = workloads.make(name)
    P = oracle.Problem(p)
    y0 = P.init_state()["y"] * 1.01     # a generic (non fixed-point) initial dual
    L, gd, gx = oracle.grad_fixed_y0(p, K, y0)
    assert L == pytest.approx(oracle.loss_fixed_y0(p, K, y0), rel=1e-12)
    rng = np.random.default_rng(1)
    big = np.argsort(-np.abs(gd))[:4]
    idx = list(big) + list(rng.choice(len(gd), 4, replace=False))

    def L_of(key, i, hh):
        q = dict(p)
        arr = p[key].copy(); arr.flat[i] += hh; q[key] = arr
        return oracle.loss_fixed_y0(q, K, y0)

    scale = max(np.abs(gd).max(), np.abs(gx).max())
    for i in idx:
        f = (L_of("obs_d", i, h) - L_of("obs_d", i, -h)) / (2 * h)
        assert abs(gd[i] - f) <= 1e-4 * abs(f) + 1e-5 * scale + floor, (i, gd[i], f)
    for i in range(p["n_s"]):
        f = (L_of("x0", i, h) - L_of("x0", i, -h)) / (2 * h)
        assert abs(gx.flat[i] - f) <= 1e-4 * abs(f) + 1e-5 * scale + floor, (i, gx.flat[i], f)
    # random unit directions over all offsets
    for _ in range(2):
        v = rng.normal(size=len(gd))
        v /= np.linalg.norm(v)
        q = dict(p); q["obs_d"] = p["obs_d"] + h * v; Lp = oracle.loss_fixed_y0(q, K, y0)
        q["obs_d"] = p["obs_d"] - h * v; Lm = oracle.loss_fixed_y0(q, K, y0)
        f = (Lp - Lm) / (2 * h)
        assert abs(gd @ v - f) <= 1e-4 * abs(f) + 1e-5 * scale + floor


def test_reverse_at_given_iterates_is_the_same_reverse_pass():
    """grad_at_iterates (the reverse pass at caller-supplied forward iterates)
    fed with the oracle's own iterates gives grad_fixed_y0 exactly, and fed
    with iterates of another run it gives that run's own gradient: the
    forward iterates are its only input besides the problem."""
    p = workloads.make("c1")
    K = 6
    y0 = oracle.Problem(p).init_state()["y"] * 1.01
    q = dict(p)
    q["eps_pri"] = -1.0
    q["eps_dual"] = -1.0
    P = oracle.Problem(q)
    st = P.init_state()
    st["y"][:] = y0
    its = [{k: v.copy() for k, v in st.items()}]
    for _ in range(K):
        P.run(st, 1)
        its.append({k: v.copy() for k, v in st.items()})
    L, gd, gx = oracle.grad_fixed_y0(p, K, y0)
    L2, gd2, gx2 = oracle.grad_at_iterates(p, its)
    assert L2 == L
    assert np.array_equal(gd2, gd) and np.array_equal(gx2, gx)
    # a different run (other initial duals): the gradient follows its iterates
    y1 = y0 * 1.05
    st = P.init_state()
    st["y"][:] = y1
    its1 = [{k: v.copy() for k, v in st.items()}]
    for _ in range(K):
        P.run(st, 1)
        its1.append({k: v.copy() for k, v in st.items()})
    _, gd3, gx3 = oracle.grad_fixed_y0(p, K, y1)
    _, gd4, gx4 = oracle.grad_at_iterates(p, its1)
    assert np.array_equal(gd3, gd4) and np.array_equal(gx3, gx4)
    assert not np.allclose(gd3, gd)
