"""GPU parity of the trajectory QP with state and input bounds (Sec. IV-A eq.
MPC_opt_origin, state and control rows; the indicator IC_0 of Sec. IV-B eq.
ADMM_Lagrangian), through the C ABI, against the FP64 oracle.

The bounded workload (c2b) is the C2 scene with speed, acceleration and
steering bounds; in the oracle's run 2 to 27 bounds are active from
iteration 2 on, and one stays active at the solution. Bars as in
test_gpu_parity: trajectories 1e-4 (normwise), duals 1e-5 per pair (scaled),
the element-wise deviation and input measures 1e-3 in 2D; the bounds are
held to 2e-6 of their size (the kernel's activation tolerance) and the set of
bounds at equality is the oracle's. Both sides start from the shared iterate
rounded to FP32."""
import numpy as np
import pytest

import oracle
import workloads
from _util import scaled_y_errors, traj_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_TRAJ = 1e-4
TOL_DUAL = 1e-5


@pytest.fixture(scope="module")
def cadmm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2406_07048_amd as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)


def gpu_state(h):
    st = h.get_state()
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in st.items()}


def fp32(st):
    return {a: np.asarray(v, np.float32).astype(np.float64) for a, v in st.items()}


def dev_errors(prob, g, o):
    xr = np.asarray(prob["x_ref"]).reshape(o["x"].shape)
    ed = eu = 0.0
    for s in range(o["x"].shape[0]):
        do = (o["x"][s] - xr[s])[1:]
        ed = max(ed, np.linalg.norm((g["x"][s] - xr[s])[1:] - do) / max(np.linalg.norm(do), 1e-300))
        eu = max(eu, np.linalg.norm(g["u"][s] - o["u"][s]) / max(np.linalg.norm(o["u"][s]), 1e-300))
    return ed, eu


def limits(prob):
    lo = np.concatenate([prob["s_min"], prob["u_min"]])
    hi = np.concatenate([prob["s_max"], prob["u_max"]])
    return lo, hi


def stage_values(st, s):
    """(x_t, u_{t-1}) stacked per step t = 1..N."""
    return np.concatenate([st["x"][s, 1:], st["u"][s]], axis=1)


def bound_report(prob, st, rel_tol):
    """Largest violation relative to max(1, |bound|), and the set of (t, k,
    side) at equality within rel_tol of the bound's size."""
    lo, hi = limits(prob)
    scale_lo = np.maximum(1.0, np.abs(np.where(np.isfinite(lo), lo, 0.0)))
    scale_hi = np.maximum(1.0, np.abs(np.where(np.isfinite(hi), hi, 0.0)))
    viol, act = 0.0, set()
    for s in range(st["x"].shape[0]):
        z = stage_values(st, s)
        viol = max(viol, np.max((lo - z) / scale_lo), np.max((z - hi) / scale_hi))
        for t, k in zip(*np.nonzero(np.abs(z - lo) <= rel_tol * scale_lo)):
            act.add((s, t, k, -1))
        for t, k in zip(*np.nonzero(np.abs(z - hi) <= rel_tol * scale_hi)):
            act.add((s, t, k, 1))
    return viol, act


_CACHE = {}


def oracle_at(prob, name, k):
    key = (name, k)
    if key not in _CACHE:
        P = oracle.Problem(prob)
        st = P.init_state()
        if k:
            P.run(st, k)
        _CACHE[key] = {a: v.copy() for a, v in st.items()}
    return oracle.Problem(prob), {a: v.copy() for a, v in _CACHE[key].items()}


def test_bounded_initial_iterate(cadmm):
    """Setup: the bounded obstacle-free trajectory equals the oracle's."""
    prob = workloads.make("c2b")
    say("[bounds] c2b initial iterate")
    h = cadmm.Handle(prob)
    g = gpu_state(h)
    h.close()
    P, st = oracle_at(prob, "c2b", 0)
    et = traj_error(g, st)
    viol, _ = bound_report(prob, g, 0)
    say(f"   traj {et:.2e} bound violation {viol:.1e}")
    assert et <= TOL_TRAJ
    assert viol <= 2e-6


@pytest.mark.parametrize("k", [1, 2, 10, 40, 80, 140])
def test_bounded_one_step(cadmm, k):
    """One GPU iteration from a shared oracle iterate equals one oracle
    iteration with bounds active (2 to 27 of them)."""
    prob = workloads.make("c2b")
    say(f"[bounds one step] c2b from iterate {k}")
    P, st64 = oracle_at(prob, "c2b", k)
    st = fp32(st64)
    h = cadmm.Handle(prob)
    h.set_state(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"])
    h.iterate(1)
    g = gpu_state(h)
    h.close()
    xk = st["x"].copy()
    P.run(st, 1)
    et = traj_error(g, st)
    ey = scaled_y_errors(prob, xk, g["y"], st["y"])
    ed, eu = dev_errors(prob, g, st)
    viol, act_g = bound_report(prob, g, 1e-5)
    _, act_o = bound_report(prob, st, 1e-9)
    say(f"   traj {et:.2e} dev {ed:.2e} u {eu:.2e} y worst {ey.max():.2e}; bounds: violation {viol:.1e}, "
        f"active {len(act_o)} (oracle) {len(act_g)} (GPU, within 1e-5)")
    assert et <= TOL_TRAJ
    assert ey.max() <= TOL_DUAL
    assert ed <= 1e-3 and eu <= 1e-3
    assert viol <= 2e-6
    assert act_o <= act_g


def test_bounded_run(cadmm):
    """60 iterations from the oracle's initial iterate stay within the
    trajectory bar, every 20 iterations; the bounds hold throughout."""
    prob = workloads.make("c2b")
    say("[bounds run] c2b 60 iterations")
    P, st = oracle_at(prob, "c2b", 0)
    h = cadmm.Handle(prob)
    h.set_state(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"])
    for k in (20, 40, 60):
        h.iterate(20)
        g = gpu_state(h)
        P.run(st, 20)
        et = traj_error(g, st)
        viol, act_g = bound_report(prob, g, 1e-5)
        _, act_o = bound_report(prob, st, 1e-9)
        say(f"   k={k}: traj err {et:.2e}, bound violation {viol:.1e}, active {len(act_o)} / {len(act_g)}")
        assert et <= TOL_TRAJ
        assert viol <= 2e-6
    h.close()


def test_bounded_solve_reports_active_bounds(cadmm):
    """admm_solve to the stopping test: every scenario's status is a count
    (no infeasible or capacity report), the trajectory holds the bounds, and
    it is the oracle's solution within the trajectory bar."""
    prob = workloads.make("c2b")
    say("[bounds solve] c2b to the stopping test")
    h = cadmm.Handle(prob)
    code, res = h.solve(300, check_every=1)
    g = gpu_state(h)
    h.close()
    P, st = oracle_at(prob, "c2b", 0)
    hist = P.run(st, 300)
    viol, act_g = bound_report(prob, g, 1e-5)
    et = traj_error(g, st)
    say(f"   GPU {res[0]['iters']} iterations, oracle {hist['iters'][0]}; active bounds {res[0]['active_bounds']}; "
        f"traj err {et:.2e}; violation {viol:.1e}")
    assert res[0]["active_bounds"] >= 0
    assert viol <= 2e-6
    assert abs(res[0]["iters"] - hist["iters"][0]) <= 3
    assert et <= TOL_TRAJ


def small_bounded_batch():
    """Three scenarios of the batched workload with speed and steering
    bounds that the manoeuvres reach."""
    p = workloads.select_scenarios(workloads.make("c4"), [0, 1, 2])
    inf = np.inf
    p.update(s_min=np.array([-inf, -inf, -inf, 7.9]), s_max=np.array([inf, inf, inf, 8.2]),
             u_min=np.array([-2.0, -0.08]), u_max=np.array([1.0, 0.08]))
    return p


def test_bounded_batched_equals_separate(cadmm):
    """Batched scenarios with bounds give bit-identical iterates to separate
    handles, and one step of the batch matches the oracle."""
    prob = small_bounded_batch()
    say("[bounds batched] 3 scenarios of c4 with bounds, 12 iterations")
    h = cadmm.Handle(prob, waves_per_group=1, lanes_per_pair=1)
    h.iterate(12)
    g = gpu_state(h)
    h.close()
    xs = []
    for s in range(3):
        q = workloads.select_scenarios(prob, [s])
        for key in ("s_min", "s_max", "u_min", "u_max"):
            q[key] = prob[key]
        hs = cadmm.Handle(q, waves_per_group=1, lanes_per_pair=1)
        hs.iterate(12)
        xs.append(gpu_state(hs)["x"][0])
        hs.close()
    assert all(np.array_equal(g["x"][s], xs[s]) for s in range(3))
    P = oracle.Problem(prob)
    st = fp32(P.init_state())
    P.run(st, 6)
    st = fp32(st)
    h = cadmm.Handle(prob)
    h.set_state(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"])
    h.iterate(1)
    g = gpu_state(h)
    h.close()
    P.run(st, 1)
    et = traj_error(g, st)
    viol, act_g = bound_report(prob, g, 1e-5)
    _, act_o = bound_report(prob, st, 1e-9)
    say(f"   one step from iterate 6: traj {et:.2e}, violation {viol:.1e}, active {len(act_o)} / {len(act_g)}")
    assert et <= TOL_TRAJ and viol <= 2e-6
    assert act_o <= act_g


def test_bounds_refuse_the_reverse_pass(cadmm):
    prob = workloads.make("c2b")
    h = cadmm.Handle(prob)
    with pytest.raises(Exception):
        h.grad_workspace_size(10, 5)
    h.close()
