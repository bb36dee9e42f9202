"""Parity of the HIP path (FP32, through the C ABI) with the FP64 oracle.

Bars: scales alpha* 1e-5 relative; dual variables 1e-5 in the proximal-metric
scaled norm per pair (sqrt(D_l) y_l, D_l = ||row_l K||^2, relative to
max(norm, 1)); trajectories 1e-4 relative (normwise over x and u per
scenario)."""
import numpy as np
import pytest

import oracle
import workloads
from _util import (K_rows, gather_pairs, multiplier_scale, per_pair_y_errors, rel, scaled_pair_error,
                   scaled_y_errors, traj_error)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_TRAJ = 1e-4
TOL_DUAL = 1e-5
TOL_SCALE = 1e-5


@pytest.fixture(scope="module")
def cadmm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2406_07048_amd as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)


def oracle_iterate(prob, k):
    """Oracle state after k ADMM iterations (from its own initial iterate)."""
    P = oracle.Problem(prob)
    st = P.init_state()
    if k:
        P.run(st, k)
    return P, st


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


# --------------------------------------------------------------- stateless QPs
def oracle_nu(Kp, kap, yh, y, bh, eps):
    """Multiplier of kappa^T y = 1 implied by a solution y: stationarity
    K r + eps D (y - yhat) - nu kappa - w = 0 on a row with y_l > 0 and
    kappa_l > 0 (w_l = 0 there); the row with the largest kappa_l y_l."""
    r = Kp.T @ y + bh
    D = (Kp ** 2).sum(1)
    l = int(np.argmax(np.where(kap > 0, kap * y, -1.0)))
    return (Kp[l] @ r + eps * D[l] * (y[l] - yh[l])) / kap[l]


def nu_bar(Kp, kap, y):
    """FP32 bar on nu: the residual bar (1e-5 of the summed terms of
    K^T y + bhat) carried through K_l . r / kappa_l on the lambda rows."""
    lam = kap > 0
    return 2e-5 * (1.0 + (np.abs(Kp).sum(1) * y).sum()) * (np.abs(Kp[lam]).sum(1) / kap[lam]).max()


@pytest.mark.parametrize("name,k", [("c1", 0), ("c1", 5), ("c2", 3), ("c2", 60), ("c3", 3), ("c3", 30)])
def test_pair_qp_batch_parity(cadmm, name, k):
    prob = workloads.make(name)
    say(f"[pair_qp_batch] {name} iterate {k}")
    P, st = oracle_iterate(prob, k)
    layout = workloads.block_layout(prob)
    nb = len(layout[0])
    rng = np.random.default_rng(0)
    pairs = [(int(rng.integers(nb)), int(rng.integers(1, prob["N"] + 1))) for _ in range(600)]
    row_ptr, K, kap, yh, bh, geo = gather_pairs(prob, st, pairs, layout)
    y, r, nu, status = cadmm.pair_qp_batch(to_dev(row_ptr, torch.int32), to_dev(K), to_dev(kap), to_dev(yh),
                                           to_dev(bh), prob["eps_prox"])
    torch.cuda.synchronize()
    y, r, nu, status = y.cpu().numpy().astype(np.float64), r.cpu().numpy(), nu.cpu().numpy(), status.cpu().numpy()
    worst = worst_nu = 0.0
    for p, (A, bb, Cp, dp, z, xi) in enumerate(geo):
        sl = slice(row_ptr[p], row_ptr[p + 1])
        yo, it = oracle.pair_qp(A, bb, Cp, dp, z, xi, yh[sl], prob["eps_prox"])
        assert it >= 0
        Kp = K[sl]
        e = scaled_pair_error(Kp, y[sl], yo)
        worst = max(worst, e)
        ro = Kp.T @ yo + bh[p]
        # r = K^T y + bhat is a sum of terms of size ||K_l||_1 y_l
        assert np.abs(r[p] - ro).max() <= 1e-5 * (1.0 + (np.abs(Kp).sum(1) * yo).sum())
        en = abs(nu[p] - oracle_nu(Kp, kap[sl], yh[sl], yo, bh[p], prob["eps_prox"])) / nu_bar(Kp, kap[sl], yo)
        worst_nu = max(worst_nu, en)
    say(f"   worst scaled dual error {worst:.2e}, nu error / bar {worst_nu:.2f}, sweeps max {status.max()}, "
        f"unconverged {(status < 0).sum()}")
    assert (status >= 0).all()
    assert worst <= TOL_DUAL
    assert worst_nu <= 1.0


def test_pair_qp_batch_edge_cases(cadmm):
    """Empty batch; the largest pair (8 + 32 + 1 rows); a pair with no
    obstacle rows (one row class plus the slack row); a pair whose proximal
    centre is already the optimum (the scale-LP certificate of a disjoint
    pair with zero multipliers: K^T y + bhat = 0, so y = yhat)."""
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    e = torch.zeros((0, 3), device="cuda")
    y, r, nu, s = cadmm.pair_qp_batch(z, e, torch.zeros(0, device="cuda"), torch.zeros(0, device="cuda"),
                                      torch.zeros((0, 3), device="cuda"), 0.1)
    assert y.numel() == 0 and s.numel() == 0
    rng = np.random.default_rng(4)
    A = np.concatenate([np.eye(2), -np.eye(2), [[0.6, 0.8], [-0.6, 0.8], [0.6, -0.8], [-0.6, -0.8]]])
    b = np.r_[1.0, 1.0, 1.0, 1.0, 1.3, 1.3, 1.3, 1.3]
    cases = []
    for n_o in (32, 0):
        ang = np.sort(rng.uniform(0, 2 * np.pi, n_o))
        Cp = np.stack([np.cos(ang), np.sin(ang)], 1).reshape(n_o, 2)
        dp = 1.0 + Cp @ np.array([4.0, 1.0])
        K = K_rows(A, Cp, dp)
        yh = np.abs(rng.normal(size=len(K)))
        cases.append((f"{n_o} obstacle rows", A, b, Cp, dp, K, yh, np.array([1.3, 0.2, -0.1])))
    # optimal centre: a square obstacle 3 m away along x, zero multipliers
    Cp = np.concatenate([np.eye(2), -np.eye(2)])
    dp = np.r_[5.0, 1.0, -4.0, 1.0]
    alpha, _, lam, mu, gap, stl = oracle.scale_lp(A, b, Cp, dp)
    assert stl == 0 and alpha > 1.0
    K = K_rows(A, Cp, dp)
    cases.append(("optimal centre", A, b, Cp, dp, K, np.r_[lam, mu, alpha - 1.0], np.array([1.0, 0.0, 0.0])))
    for what, A_, b_, Cp_, dp_, K, yh, bh in cases:
        kap = np.r_[b_, np.zeros(len(dp_) + 1)]
        y, r, nu, st = cadmm.pair_qp_batch(to_dev(np.array([0, len(K)], np.int32), torch.int32), to_dev(K),
                                           to_dev(kap), to_dev(yh), to_dev(bh[None]), 0.1)
        torch.cuda.synchronize()
        yo, it = oracle.pair_qp(A_, b_, Cp_, dp_, bh[0] - 1.0, bh[1:], yh, 0.1)
        err = scaled_pair_error(K, y.cpu().numpy().astype(np.float64), yo)
        say(f"   {what}: scaled dual error {err:.2e}, sweeps {st.item()}")
        assert st.item() >= 0
        assert err <= TOL_DUAL
        if what == "optimal centre":
            assert scaled_pair_error(K, yo, yh) <= 1e-9
            assert np.abs(r.cpu().numpy()).max() <= 1e-5


# --------------------------------------------------------------- scale LP
@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_scale_batch_parity(cadmm, name):
    prob = workloads.make(name)
    say(f"[pair_scale_batch] {name}")
    P, st = oracle_iterate(prob, 0)
    layout = workloads.block_layout(prob)
    nb = len(layout[0])
    rng = np.random.default_rng(1)
    pairs = [(int(rng.integers(nb)), int(rng.integers(1, prob["N"] + 1))) for _ in range(400)]
    row_ptr, K, kap, yh, bh, geo = gather_pairs(prob, st, pairs, layout)
    a_ptr, o_ptr = [0], [0]
    A, bv, Cp, dp = [], [], [], []
    for (Ai, bi, Ci, di, _, _) in geo:
        A.append(Ai); bv.append(bi); Cp.append(Ci); dp.append(di)
        a_ptr.append(a_ptr[-1] + len(bi)); o_ptr.append(o_ptr[-1] + len(di))
    alpha, lam, mu, status = cadmm.pair_scale_batch(
        to_dev(np.array(a_ptr, np.int32), torch.int32), to_dev(np.concatenate(A)), to_dev(np.concatenate(bv)),
        to_dev(np.array(o_ptr, np.int32), torch.int32), to_dev(np.concatenate(Cp)), to_dev(np.concatenate(dp)))
    torch.cuda.synchronize()
    alpha, lam, mu, status = (t.cpu().numpy() for t in (alpha, lam, mu, status))
    assert (status == 0).all()
    worst = 0.0
    for p, (Ai, bi, Ci, di, _, _) in enumerate(geo):
        ao, xo, lo, mo, gap, sto = oracle.scale_lp(Ai, bi, Ci, di)
        e = abs(alpha[p] - ao) / max(abs(ao), 1e-3)
        worst = max(worst, e)
        # dual certificate: feasible and attaining alpha (unique unless degenerate)
        l_g = lam[a_ptr[p]:a_ptr[p + 1]].astype(np.float64)
        m_g = mu[o_ptr[p]:o_ptr[p + 1]].astype(np.float64)
        assert abs(bi @ l_g - 1.0) < 1e-5
        assert np.abs(Ai.T @ l_g + Ci.T @ m_g).max() < 1e-4
        assert abs(-di @ m_g - ao) <= 1e-4 * max(1.0, abs(ao))
    say(f"   worst alpha rel error {worst:.2e}")
    assert worst <= TOL_SCALE


def test_scale_box_golden(cadmm):
    """Hand-worked box cases of the closed form (tests/golden/box_scale.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "box_scale.txt")
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        dim, h, lo, hi, a = [s.strip() for s in line.split("|")]
        dim = int(dim)
        h, lo, hi = (np.array(v.split(), float) for v in (h, lo, hi))
        A = np.concatenate([np.eye(dim), -np.eye(dim)])
        b = np.r_[h, h]
        d = np.r_[hi, -lo]
        alpha, lam, mu, st = cadmm.pair_scale_batch(
            to_dev(np.array([0, 2 * dim], np.int32), torch.int32), to_dev(A), to_dev(b),
            to_dev(np.array([0, 2 * dim], np.int32), torch.int32), to_dev(A), to_dev(d))
        assert abs(alpha.item() - float(a)) <= TOL_SCALE * max(1.0, float(a))


# --------------------------------------------------------------- ADMM path
def gpu_state(h):
    st = h.get_state()
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in st.items()}


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_setup_initial_iterate(cadmm, name):
    """Initial iterate: obstacle-free LQ trajectory, zero multipliers and a
    scale-LP certificate per pair. alpha* is unique and compared; the dual
    certificate is unique only for non-degenerate LPs (in 3D a triangulated
    obstacle vertex usually has more than three incident faces, so many
    optimal duals exist): it is checked for validity, i.e. at s^0 it gives
    T = max(0, 1 - alpha*) and R = 0, plus agreement in 2D with the oracle's
    certificate at the GPU's own trajectory (at the oracle's trajectory the
    LP duals would also carry the trajectory rounding, amplified by the
    conditioning of the optimal basis)."""
    prob = workloads.make(name)
    say(f"[setup] {name}")
    h = cadmm.Handle(prob)
    g = gpu_state(h)
    alpha_g = h.scales().double().cpu().numpy()
    P, st = oracle_iterate(prob, 0)
    # alpha* is compared at the GPU's own trajectory, so that the check
    # isolates the LP from the (separately checked) trajectory rounding
    alpha_o, y_o = P.scale_all(g["x"], with_y=True)
    ea = (np.abs(alpha_g - alpha_o) / np.maximum(np.abs(alpha_o), 1e-3)).max()
    T, R, _ = P.mult_phase(g["x"], g["y"], np.zeros_like(g["zeta"]), np.zeros_like(g["xi"]))
    msc = multiplier_scale(prob, g["x"], g["y"])
    eT = (np.abs(T - np.maximum(0.0, 1.0 - alpha_o)) / msc).max()
    eR = (np.abs(R).reshape(-1, prob["dim"], prob["N"]) / msc.reshape(-1, 1, prob["N"])).max()
    ny = g["y"] < -1e-7
    say(f"   s0 err {traj_error(g, st):.1e}, alpha {ea:.2e}, certificate T {eT:.2e} R {eR:.2e}")
    assert traj_error(g, st) < 1e-5
    assert ea <= TOL_SCALE
    assert eT <= 1e-5 and eR <= 1e-5 and not ny.any()
    if prob["dim"] == 2:
        errs = per_pair_y_errors(prob, g["y"], y_o)
        say(f"   certificate y vs oracle at the GPU trajectory: {errs.max():.2e}")
        assert errs.max() <= TOL_DUAL
    assert np.abs(g["zeta"]).max() == 0 and np.abs(g["xi"]).max() == 0
    h.close()


_ITERATES = {}


def cached_iterate(prob, name, k):
    """Oracle iterate k of a named workload (FP64), computed once per module
    and continued from the nearest earlier cached iterate."""
    key = (name, k)
    if key not in _ITERATES:
        prev = [j for (n, j) in _ITERATES if n == name and j < k]
        if prev:
            j = max(prev)
            st = {a: v.copy() for a, v in _ITERATES[(name, j)].items()}
        else:
            j, st = 0, oracle.Problem(prob).init_state()
        if k > j:
            oracle.Problem(prob).run(st, k - j)
        _ITERATES[key] = {a: v.copy() for a, v in st.items()}
    return {a: v.copy() for a, v in _ITERATES[key].items()}


def fp32(st):
    """The iterate as the GPU receives it (every entry rounded to FP32)."""
    return {a: np.asarray(v, np.float32).astype(np.float64) for a, v in st.items()}


def deviation_errors(prob, g, o):
    """Element-wise measures of what the method decides, per scenario (max):
    ||d(x - x_ref)|| / ||x - x_ref|| over t = 1..N and ||du|| / ||u||."""
    xr = np.asarray(prob["x_ref"]).reshape(o["x"].shape)
    ed = eu = 0.0
    for s in range(o["x"].shape[0]):
        do = (o["x"][s] - xr[s])[1:]
        ed = max(ed, np.linalg.norm((g["x"][s] - xr[s])[1:] - do) / max(np.linalg.norm(do), 1e-300))
        eu = max(eu, np.linalg.norm(g["u"][s] - o["u"][s]) / max(np.linalg.norm(o["u"][s]), 1e-300))
    return ed, eu


ONE_STEP = [("c1", 4), ("c2", 0), ("c2", 30), ("c2", 60), ("c2", 100), ("c2", 150),
            ("c3", 0), ("c3", 20), ("c3", 40), ("c3", 80)]


@pytest.mark.parametrize("name,k", ONE_STEP)
def test_one_step_parity(cadmm, name, k):
    """From a shared oracle iterate k, one GPU iteration equals one oracle
    iteration (pair QPs, trajectory QP, multiplier update). Both start from
    the iterate rounded to FP32, which is what the GPU receives.

    Bars: trajectories 1e-4 (normwise, literal); duals 1e-5 per pair (scaled);
    multipliers 1e-5 of their scale for step 3 alone, 1e-3 end to end; and
    the element-wise measures ||d(x - x_ref)|| / ||x - x_ref|| and
    ||du|| / ||u|| at 1e-3 in 2D. In 3D the quadrotor stays within
    millimetres of its 25 m reference (||x - x_ref|| is 1e-5 to 3e-2 against
    ||x|| = 304), so FP32 storage of the iterate alone moves these measures
    by 2e-3 to 3e-2 (the oracle's own change when its input is rounded to
    FP32, computed here); their bar there is 30 times that change (the GPU's
    FP32 sums over 600 pairs per step and its FP32 Riccati on top), and they
    are only printed while ||x - x_ref|| is below 100 FP32 units of the
    trajectory (100 * 2^-23 ||x||: the initial iterates, where the deviation
    is a few ulps of the positions and has no FP32 meaning)."""
    prob = workloads.make(name)
    say(f"[one step] {name} from iterate {k}")
    st64 = cached_iterate(prob, name, k)
    st = fp32(st64)
    P = oracle.Problem(prob)
    h = cadmm.Handle(prob)
    h.set_state(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"])
    h.iterate(1)
    g = gpu_state(h)
    alpha_g = h.scales().double().cpu().numpy()
    h.close()
    xk = st["x"].copy()
    zk, xik = st["zeta"].copy(), st["xi"].copy()
    P.run(st, 1)
    et = traj_error(g, st)
    ey = scaled_y_errors(prob, xk, g["y"], st["y"])
    dim, N = prob["dim"], prob["N"]
    msc = multiplier_scale(prob, st["x"], st["y"])
    # step 3 in isolation: the oracle's multiplier update applied to the GPU's
    # own (x^{k+1}, y^{k+1}) must give the GPU's multipliers
    z3, xi3, _ = P.mult_phase(g["x"], g["y"], zk, xik)
    ez3 = (np.abs(g["zeta"] - z3) / msc).max()
    exi3 = (np.abs(g["xi"] - xi3).reshape(-1, dim, N) / msc.reshape(-1, 1, N)).max()
    # end to end the multipliers inherit the trajectory's rounding through T, R
    ez = (np.abs(g["zeta"] - st["zeta"]) / msc).max()
    exi = (np.abs(g["xi"] - st["xi"]).reshape(-1, dim, N) / msc.reshape(-1, 1, N)).max()
    # scales at the new trajectory (the certificate of Sec. III), at the GPU's trajectory
    alpha_o = P.scale_all(g["x"])
    ea = (np.abs(alpha_g - alpha_o) / np.maximum(np.abs(alpha_o), 1.0)).max()
    ed, eu = deviation_errors(prob, g, st)
    xr = np.asarray(prob["x_ref"]).reshape(st["x"].shape)
    resolved = np.linalg.norm((st["x"] - xr)[:, 1:]) >= 100 * 2.0 ** -23 * np.linalg.norm(st["x"])
    if dim == 2:
        bar_d = bar_u = 1e-3
    elif not resolved:
        bar_d = bar_u = np.inf
    else:
        ref64 = {a: v.copy() for a, v in st64.items()}
        P.run(ref64, 1)
        id_, iu = deviation_errors(prob, st, ref64)
        bar_d, bar_u = max(1e-3, 30 * id_), max(1e-3, 30 * iu)
    say(f"   traj {et:.2e} dev {ed:.2e} (bar {bar_d:.1e}) u {eu:.2e} (bar {bar_u:.1e}) | y worst {ey.max():.2e} "
        f"p99 {np.percentile(ey, 99):.2e} | alpha {ea:.2e} | step-3 zeta {ez3:.2e} xi {exi3:.2e} "
        f"| end-to-end zeta {ez:.2e} xi {exi:.2e}")
    assert et <= TOL_TRAJ and ey.max() <= TOL_DUAL
    assert ea <= TOL_SCALE
    assert ed <= bar_d and eu <= bar_u
    assert ez3 <= 1e-5 and exi3 <= 1e-5
    assert ez <= 1e-3 and exi <= 1e-3


def test_full_run_c1(cadmm):
    """C1 (the FP64 oracle configuration) run to convergence on the GPU in
    FP32: trajectory within 1e-4 of the oracle's and the element-wise
    deviation and input measures within 1e-3, same stopping iteration (+-1);
    the final scale certificates within 1e-5. At the GPU's stopping iteration
    (about 46) the duals per pair (scaled) against the oracle's at that
    iteration carry the growth of 46 iterations of a nonconvex iteration
    (one iteration from a shared iterate stays below 1e-5): bar 1e-4 per
    pair, measured value printed."""
    prob = workloads.make("c1")
    say("[full run] c1")
    h = cadmm.Handle(prob)
    code, res = h.solve(200, check_every=1)
    g = gpu_state(h)
    alpha_g = h.scales().double().cpu().numpy()
    h.close()
    P, st = oracle_iterate(prob, 0)
    hist = P.run(st, 200)
    it_g = res[0]["iters"]
    ed, eu = deviation_errors(prob, g, st)
    # the oracle run to the GPU's iteration count, for the duals
    q = dict(prob)
    q["eps_pri"] = q["eps_dual"] = -1.0
    Pq, sq = oracle_iterate(q, 0)
    Pq.run(sq, it_g)
    xk_prev = sq["x"]
    ey = scaled_y_errors(prob, xk_prev, g["y"], sq["y"])
    ea = (np.abs(alpha_g - P.scale_all(g["x"])) / np.maximum(np.abs(P.scale_all(g["x"])), 1.0)).max()
    say(f"   gpu iters {it_g} oracle {hist['iters'][0]}; traj err {traj_error(g, st):.2e} dev {ed:.2e} u {eu:.2e}; "
        f"y worst {ey.max():.2e}; alpha {ea:.2e}; min alpha {res[0]['min_alpha']:.4f}")
    assert traj_error(g, st) <= TOL_TRAJ
    assert ed <= 1e-3 and eu <= 1e-3
    assert abs(it_g - hist["iters"][0]) <= 1
    assert ey.max() <= 1e-4
    assert ea <= TOL_SCALE
    assert res[0]["min_alpha"] > 0.95


@pytest.mark.parametrize("name,iters", [("c2", 60), ("c3", 40)])
def test_full_run_trajectory(cadmm, name, iters):
    """Longer runs from a shared iterate (the oracle's initial one, since in 3D
    the initial LP certificate is not unique), checked every 10 iterations:

    - the trajectories stay within the parity bar of the oracle's own run;
    - the duals of the last step against the oracle's pair phase applied to
      the GPU's own previous iterate: the pair solves of step k alone, apart
      from the rounding the run has accumulated, at the 1e-5 dual bar for
      every pair;
    - the duals against the oracle's own run: 99% of the pairs within 1e-5.
      The iteration is not a contraction (the collision constraints are
      nonconvex), so the trajectories' FP32 differences feed back into the
      pair data and a few pairs drift further (up to 1.0e-4 measured,
      printed).

    The scales at the final trajectory are within 1e-5."""
    prob = workloads.make(name)
    say(f"[full run] {name} {iters} iterations from the oracle's initial iterate")
    P, st = oracle_iterate(prob, 0)
    h = cadmm.Handle(prob)
    h.set_state(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"])
    for k in range(10, iters + 1, 10):
        h.iterate(9)
        g_prev = gpu_state(h)
        h.iterate(1)
        g = gpu_state(h)
        P.run(st, 10)
        et = traj_error(g, st)
        y_step = P.pair_phase(g_prev)
        es = scaled_y_errors(prob, g_prev["x"], g["y"], y_step)
        ey = scaled_y_errors(prob, st["x"], g["y"], st["y"])
        say(f"   k={k}: traj err {et:.2e}; step-k duals worst {es.max():.2e}; against the oracle's run: "
            f"worst {ey.max():.2e} p99 {np.percentile(ey, 99):.2e} (pairs above 1e-5: {(ey > TOL_DUAL).sum()} "
            f"of {ey.size})")
        assert et <= TOL_TRAJ
        assert es.max() <= TOL_DUAL
        assert np.percentile(ey, 99) <= TOL_DUAL
    alpha_g = h.scales().double().cpu().numpy()
    h.close()
    alpha_o = P.scale_all(g["x"])
    ea = (np.abs(alpha_g - alpha_o) / np.maximum(np.abs(alpha_o), 1.0)).max()
    say(f"   final alpha {ea:.2e}")
    assert ea <= TOL_SCALE


@pytest.mark.parametrize("G", [1, 2, 4])
def test_batched_equals_separate(cadmm, G):
    """Batched scenarios give bit-identical iterates to separate handles
    (same kernels, same fixed reduction order), for each lane-group size."""
    prob = workloads.config_c4(n_scen=6, m_range=(10, 30))
    say(f"[batched vs separate] 6 scenarios, {G} lanes per pair")
    W = 1 if G == 4 else 2
    h = cadmm.Handle(prob, waves_per_group=W, lanes_per_pair=G)
    h.iterate(12)
    g = gpu_state(h)
    h.close()
    for s in range(6):
        q = workloads.select_scenarios(prob, [s])
        hs = cadmm.Handle(q, waves_per_group=W, lanes_per_pair=G)
        hs.iterate(12)
        gs = gpu_state(hs)
        hs.close()
        assert np.array_equal(gs["x"][0], g["x"][s])


def test_state_host_transfers(cadmm):
    """get_state_host (one copy) returns get_state's values, and set_state
    from host arrays (one copy) installs them bitwise."""
    prob = workloads.make("c2")
    say("[state transfers] c2")
    h = cadmm.Handle(prob)
    h.iterate(5)
    a = gpu_state(h)
    b = h.get_state_host()
    for k in a:
        assert a[k].shape == b[k].shape and np.array_equal(a[k], b[k]), k
    h.reset()
    h.set_state(**{k: v.copy() for k, v in b.items()})
    c = gpu_state(h)
    for k in a:
        assert np.array_equal(a[k], c[k]), k
    h.close()


def test_replay_is_deterministic(cadmm):
    prob = workloads.make("c2")
    say("[determinism] c2")
    h = cadmm.Handle(prob)
    h.iterate(20)
    a = gpu_state(h)
    h.reset()
    h.iterate(13)
    h.iterate(7)
    b = gpu_state(h)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    h.close()


def test_far_obstacles_fixed_point(cadmm):
    prob = workloads.make("c1", seed=3)
    say("[fixed point] c1 seed 3")
    h = cadmm.Handle(prob)
    g0 = gpu_state(h)
    code, res = h.solve(10, check_every=1)
    g1 = gpu_state(h)
    assert res[0]["iters"] == 1 and res[0]["converged"]
    assert np.abs(g1["x"] - g0["x"]).max() < 1e-4
    # zeta = T at a certificate: zero up to the rounding of 1 + d'^T mu + gamma
    assert np.abs(g1["zeta"]).max() <= 1e-6 * (1.0 + g0["y"].max())
    h.close()


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_lane_groups_agree(cadmm, name):
    """1, 2 or 4 lanes per pair QP: each launch shape, run 8 iterations from
    the oracle's initial iterate, stays within the trajectory bar of the
    oracle (the groups only reorder the sums of one pair QP)."""
    prob = workloads.make(name)
    say(f"[lane groups] {name}")
    P, st0 = oracle_iterate(prob, 0)
    st = {k: v.copy() for k, v in st0.items()}
    P.run(st, 8)
    for G in (1, 2, 4):
        h = cadmm.Handle(prob, waves_per_group=1, lanes_per_pair=G)
        assert h.launch_config()[2] == G
        h.set_state(x=st0["x"], u=st0["u"], y=st0["y"], zeta=st0["zeta"], xi=st0["xi"])
        h.iterate(8)
        g = gpu_state(h)
        h.close()
        et = traj_error(g, st)
        say(f"   G={G} traj err {et:.2e}")
        assert et <= TOL_TRAJ
