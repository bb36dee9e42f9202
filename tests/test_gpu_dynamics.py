"""GPU parity of the dynamics beyond one time-invariant linear model, through
the C ABI, against the FP64 oracle:

- time-varying linear models (Sec. IV-A eq. system_eqn given linearised per
  step): the curved-reference workload, one model per scenario and step;
  setup (obstacle-free LQ), one step from shared oracle iterates, a longer
  run, the reverse pass at the GPU's own iterates, batched vs separate;
- the nonlinear bicycle and quadrotor relinearised about every iterate (the
  one SQP step per ADMM iteration of Sec. IV-B): one step from shared oracle
  iterates (C2 and C3 geometry), a 40-iteration run, the obstacle-free SQP
  run closing the dynamics defects, and the reverse pass refusing the
  nonlinear models.

Bars as in test_gpu_parity: trajectories 1e-4 (normwise), duals 1e-5 per
pair (scaled), the element-wise deviation and input measures 1e-3 in 2D;
both sides start from the shared iterate rounded to FP32."""
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


def oracle_at(prob, k):
    P = oracle.Problem(prob)
    st = P.init_state()
    if k:
        P.run(st, k)
    return P, st


def test_time_varying_setup(cadmm):
    """Obstacle-free LQ with one model per scenario and step, and the
    scale-LP certificates, at setup."""
    prob = workloads.make("c2tv")
    say("[tv setup] c2tv")
    h = cadmm.Handle(prob)
    g = gpu_state(h)
    alpha = h.scales().double().cpu().numpy()
    h.close()
    P, st = oracle_at(prob, 0)
    ao = P.scale_all(g["x"])
    ea = (np.abs(alpha - ao) / np.maximum(np.abs(ao), 1.0)).max()
    say(f"   s0 err {traj_error(g, st):.2e} alpha {ea:.2e}")
    assert traj_error(g, st) <= 1e-5
    assert ea <= 1e-5


@pytest.mark.parametrize("name,k", [("c2tv", 0), ("c2tv", 5), ("c2tv", 15),
                                    ("c2sqp", 0), ("c2sqp", 30), ("c2sqp", 100),
                                    ("c3sqp", 0), ("c3sqp", 20)])
def test_one_step(cadmm, name, k):
    """One GPU iteration from a shared oracle iterate equals one oracle
    iteration: time-varying models (c2tv) and the SQP step of the nonlinear
    bicycle (c2sqp) and quadrotor (c3sqp)."""
    prob = workloads.make(name)
    say(f"[dynamics one step] {name} from iterate {k}")
    P, st64 = oracle_at(prob, k)
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
    say(f"   traj {et:.2e} dev {ed:.2e} u {eu:.2e} y worst {ey.max():.2e}")
    assert et <= TOL_TRAJ
    assert ey.max() <= TOL_DUAL
    if prob["dim"] == 2:
        assert ed <= 1e-3 and eu <= 1e-3


@pytest.mark.parametrize("name,iters", [("c2tv", 20), ("c2sqp", 40), ("c3sqp", 20)])
def test_longer_run(cadmm, name, iters):
    """Runs from the oracle's initial iterate stay within the trajectory bar."""
    prob = workloads.make(name)
    say(f"[dynamics run] {name} {iters} iterations")
    P, st = oracle_at(prob, 0)
    h = cadmm.Handle(prob)
    h.set_state(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"])
    h.iterate(iters)
    g = gpu_state(h)
    h.close()
    P.run(st, iters)
    et = traj_error(g, st)
    say(f"   traj err {et:.2e}")
    assert et <= TOL_TRAJ


def test_sqp_closes_the_dynamics_defects(cadmm):
    """Without obstacles the SQP iteration on the nonlinear bicycle converges
    to a trajectory that satisfies the nonlinear dynamics, the same as the
    oracle's (stopping test off). The start is 0.3 m and 0.02 rad off the
    reference: the step has no globalisation (one QP per iteration, Sec.
    IV-B), and from 1.5 m / 0.1 rad the oracle's iteration cycles too."""
    prob = workloads.with_obstacles(workloads.make("c2sqp"), [[]])
    prob["x0"] = prob["x0"] + np.array([[0.0, 0.3, 0.02, 0.0]])
    prob["eps_pri"] = prob["eps_dual"] = -1.0
    say("[sqp defects] c2sqp without obstacles")
    h = cadmm.Handle(prob)
    h.iterate(30)
    g = gpu_state(h)
    h.close()
    P, st = oracle_at(prob, 30)
    dt, L = prob["model_par"]
    defect = max(np.abs(workloads.bicycle_step(g["x"][0, t], g["u"][0, t], dt, L) - g["x"][0, t + 1]).max()
                 for t in range(prob["N"]))
    say(f"   traj err {traj_error(g, st):.2e}, max nonlinear defect {defect:.2e}")
    assert traj_error(g, st) <= TOL_TRAJ
    assert defect <= 1e-4


def test_time_varying_batched_equals_separate(cadmm):
    """Per-scenario models: the batched run equals separate runs bitwise."""
    prob = workloads.make("c2tv")
    say("[tv batched vs separate]")
    h = cadmm.Handle(prob, waves_per_group=1, lanes_per_pair=2)
    h.iterate(6)
    g = gpu_state(h)
    h.close()
    for s in range(workloads.n_scenarios(prob)):
        q = workloads.select_scenarios(prob, [s])
        hs = cadmm.Handle(q, waves_per_group=1, lanes_per_pair=2)
        hs.iterate(6)
        gs = gpu_state(hs)
        hs.close()
        assert np.array_equal(gs["x"][0], g["x"][s])


def test_time_varying_reverse_pass(cadmm):
    """Reverse pass with one model per scenario and step: admm_backward
    against the oracle's reverse recursion at the GPU's own forward
    iterates (bars as in test_gpu_grad: offsets 1e-4, x0 1e-3)."""
    prob = workloads.make("c2tv")
    prob["eps_pri"] = prob["eps_dual"] = -1.0
    K = 8
    say(f"[tv reverse] c2tv K={K}")
    y0 = oracle.Problem(prob).init_state()["y"] * 1.01
    h = cadmm.Handle(prob)
    h.set_state(y=torch.as_tensor(y0, dtype=torch.float32))
    h.record(K, 3)
    gd, gx = h.backward(1.0)
    gd, gx = gd.double().cpu().numpy(), gx.double().cpu().numpy()
    h.reset()
    h.set_state(y=torch.as_tensor(y0, dtype=torch.float32))
    its = [gpu_state(h)]
    for _ in range(K):
        h.iterate(1)
        its.append(gpu_state(h))
    h.close()
    _, gdo, gxo = oracle.grad_at_iterates(prob, its)
    ed = np.linalg.norm(gd - gdo) / np.linalg.norm(gdo)
    ex = np.linalg.norm(gx.ravel() - gxo.ravel()) / np.linalg.norm(gxo)
    say(f"   grad_d rel {ed:.2e} grad_x0 rel {ex:.2e}")
    assert ed <= 1e-4 and ex <= 1e-3


def test_nonlinear_model_has_no_reverse_pass(cadmm):
    prob = workloads.make("c2sqp")
    h = cadmm.Handle(prob)
    with pytest.raises(cadmm.CadmmError):
        h.grad_workspace_size(5, 1)
    h.close()
