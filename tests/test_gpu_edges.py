"""GPU parity at the edges of the supported sizes and at full batched size.

- The largest compiled pair shapes: 2D with an 8-face robot part and
  obstacles of up to 32 faces, 3D with prism obstacles of 25-32 faces (the pair
  kernel variants of 8 robot rows and 32 obstacle rows).
- The horizon extremes N = 1 and N = 64 (the register Riccati sweep and the
  one-lane / full-wave pair blocks).
- The full 256-scenario batched workload, in the launch configuration the
  benchmark times (autotuned), on sampled scenarios against the oracle.

Bars as in test_gpu_parity: trajectories 1e-4 relative, duals 1e-5 in the
proximal-metric scaled norm, also for the 3D case with 25-32-face obstacles,
whose thin arm parts (b = 0.02 m) give far pairs with duals of size 30
(alpha* near 29). Both sides start from the shared iterate rounded to FP32
(what the GPU receives)."""
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


EDGE = {
    "2d-faces32-N20": lambda: workloads.config_edge_2d(N=20),
    "2d-N1": lambda: workloads.config_edge_2d(N=1),
    "2d-N64": lambda: workloads.config_edge_2d(N=64),
    "3d-faces32-N10": lambda: workloads.config_edge_3d(N=10),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_sizes_one_step(cadmm, name):
    """From a shared oracle iterate (k = 3), one GPU iteration equals one
    oracle iteration, for every lane-group size."""
    prob = EDGE[name]()
    say(f"[edge one step] {name}")
    P = oracle.Problem(prob)
    st0 = P.init_state()
    P.run(st0, 3)
    st0 = {a: np.asarray(v, np.float32).astype(np.float64) for a, v in st0.items()}
    xk = st0["x"].copy()
    ref = {k: v.copy() for k, v in st0.items()}
    P.run(ref, 1)
    for G in (1, 2, 4):
        W = 1
        h = cadmm.Handle(prob, waves_per_group=W, lanes_per_pair=G)
        h.set_state(x=st0["x"], u=st0["u"], y=st0["y"], zeta=st0["zeta"], xi=st0["xi"])
        h.iterate(1)
        g = gpu_state(h)
        h.close()
        et = traj_error(g, ref)
        ey = scaled_y_errors(prob, xk, g["y"], ref["y"])
        say(f"   G={G}: traj {et:.2e} y worst {ey.max() if ey.size else 0.0:.2e}")
        assert et <= TOL_TRAJ
        assert ey.size == 0 or ey.max() <= TOL_DUAL


@pytest.mark.parametrize("name", ["2d-faces32-N20", "2d-N64"])
def test_edge_sizes_initial_iterate(cadmm, name):
    """Setup at the edge sizes: the obstacle-free LQ trajectory and the scale
    factors match the oracle."""
    prob = EDGE[name]()
    say(f"[edge setup] {name}")
    h = cadmm.Handle(prob)
    g = gpu_state(h)
    alpha_g = h.scales().double().cpu().numpy()
    h.close()
    P = oracle.Problem(prob)
    st = P.init_state()
    alpha_o = P.scale_all(g["x"])
    ea = (np.abs(alpha_g - alpha_o) / np.maximum(np.abs(alpha_o), 1.0)).max()
    say(f"   s0 err {traj_error(g, st):.1e}, alpha {ea:.2e}")
    assert traj_error(g, st) < 1e-5
    assert ea <= 1e-5


def test_full_batched_size_sampled(cadmm):
    """All 256 batched scenarios in one autotuned handle, 8 iterations from
    the GPU's own initial iterate; three sampled scenarios (first, middle,
    last) against the oracle run on each alone."""
    prob = workloads.make("c4")
    S = workloads.n_scenarios(prob)
    say(f"[full batched size] {S} scenarios, 8 iterations")
    h = cadmm.Handle(prob)
    h.iterate(8)
    g = gpu_state(h)
    say(f"   launch shape {h.launch_config()}")
    h.close()
    for s in (0, S // 2, S - 1):
        q = workloads.select_scenarios(prob, [s])
        P = oracle.Problem(q)
        st = P.init_state()
        P.run(st, 8)
        gs = {"x": g["x"][s:s + 1], "u": g["u"][s:s + 1]}
        et = traj_error(gs, st)
        say(f"   scenario {s}: traj err {et:.2e}")
        assert et <= TOL_TRAJ
