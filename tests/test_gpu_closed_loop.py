"""The receding-horizon closed loop (Sec. V-A use: one MPC solve per control
cycle, the first input applied to a simulated plant) on the library, against
the same loop run on the FP64 oracle, through the C ABI.

The oracle's loop is written here from the same cycle rules (the sensed
obstacle set, the reference window, the warm start shifted one step with the
duals and multipliers of still-sensed obstacles carried, the nonlinear
quadrotor as plant); it shares no code with the library's driver. Both run a
fixed number of ADMM iterations per cycle (no stopping test) so that the
loops are the same map; from the same start in the obstacle-dense stretch
the predicted trajectories agree within the trajectory bar (1e-4 normwise)
every cycle, and so do the plant states they produce. A second case runs the
whole 25 s scene with the stopping test and reports the time per control
loop."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_TRAJ = 1e-4


@pytest.fixture(scope="module")
def cadmm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2406_07048_amd as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)


def oracle_loop(scene, k0, x_start, cycles, iters, carry_multipliers=True):
    """The loop on the oracle: per cycle a fresh oracle problem of the sensed
    obstacles, its initial iterate overwritten by the previous solution
    shifted one step, `iters` ADMM iterations, the first input to the plant."""
    N = scene["base"]["N"]
    dim = scene["base"]["dim"]
    x = np.array(x_start, np.float64)
    prev = None
    xs, preds = [x.copy()], []
    for k in range(k0, k0 + cycles):
        ids = workloads.sensed(scene, x[:3])
        prob = workloads.cycle_problem(scene, ids, x, k)
        prob.update(eps_pri=-1.0, eps_dual=-1.0)
        P = oracle.Problem(prob)
        st = P.init_state()
        sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
        keys = {(int(part[b]), int(ids[obs[b]])): b for b in range(len(sc))}
        if prev is not None:
            st["x"][0, 0] = x
            st["x"][0, 1:N] = prev["x"][0, 2:N + 1]
            st["x"][0, N] = prev["x"][0, N]
            st["u"][0, :N - 1] = prev["u"][0, 1:]
            st["u"][0, N - 1] = prev["u"][0, N - 1]
            # pair blocks start from the scale-LP certificates at the warm
            # trajectory; those of still-sensed obstacles from the shifted duals
            st["y"] = P.scale_all(st["x"], with_y=True)[1]
            st["zeta"][:] = 0.0
            st["xi"][:] = 0.0
            for key, b in keys.items():
                if key not in prev["keys"]:
                    continue
                ob = prev["keys"][key]
                n = int(nrow[b])
                yo = prev["y"][prev["yoff"][ob]:prev["yoff"][ob] + n * N].reshape(n, N)
                st["y"][yoff[b]:yoff[b] + n * N] = np.concatenate([yo[:, 1:], yo[:, -1:]], axis=1).ravel()
                if not carry_multipliers:
                    continue
                zo = prev["zeta"][ob * N:(ob + 1) * N]
                st["zeta"][b * N:(b + 1) * N] = np.concatenate([zo[1:], zo[-1:]])
                xo = prev["xi"][ob * dim * N:(ob + 1) * dim * N].reshape(dim, N)
                st["xi"][b * dim * N:(b + 1) * dim * N] = np.concatenate([xo[:, 1:], xo[:, -1:]], axis=1).ravel()
        P.run(st, iters)
        preds.append(st["x"][0].copy())
        x = P.model_step(x, st["u"][0, 0])[0]
        xs.append(x.copy())
        prev = dict(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"], keys=keys, yoff=yoff)
    return np.array(xs), preds


def test_closed_loop_matches_oracle_loop(cadmm):
    from paper_2406_07048_amd.closed_loop import ClosedLoop
    scene = workloads.closed_loop_scene()
    k0, cycles, iters = 120, 5, 25
    x_start = scene["ref"][k0].copy()
    say(f"[closed loop] cycles {k0}..{k0 + cycles - 1}, {iters} iterations each, from the reference at y = "
        f"{x_start[1]:.1f} m")
    loop = ClosedLoop(scene, fixed_iters=iters)
    out = loop.run(cycles, k0=k0, x_start=x_start)
    loop.close()
    xs_o, preds_o = oracle_loop(scene, k0, x_start, cycles, iters)
    for c, rec in enumerate(out["records"]):
        xp, xo = rec["x_pred"], preds_o[c]
        et = np.linalg.norm(xp - xo) / np.linalg.norm(xo)
        es = np.linalg.norm(out["x"][c + 1] - xs_o[c + 1]) / np.linalg.norm(xs_o[c + 1])
        eu = np.linalg.norm(rec["u0"] - out["u"][c]) if c < len(out["u"]) else 0.0
        say(f"   cycle {rec['k']}: sensed {rec['sensed']} ({rec['pairs']} pairs{', new set-up' if rec['setup'] else ''}); "
            f"predicted trajectory {et:.2e}, plant state {es:.2e}")
        assert et <= TOL_TRAJ
        assert es <= TOL_TRAJ
        assert eu == 0.0


def test_closed_loop_scene_run(cadmm):
    """The whole scene (250 cycles of 0.1 s) with the stopping test: every
    solve ends (within the iteration cap), the robot ends near the goal, and
    the per-cycle times are reported."""
    from paper_2406_07048_amd.closed_loop import ClosedLoop
    scene = workloads.closed_loop_scene()
    cycles = len(scene["ref"]) - 1
    say(f"[closed loop] the whole scene, {cycles} cycles with the stopping test")
    loop = ClosedLoop(scene, max_iters=100, check_every=8)
    out = loop.run(cycles)
    loop.close()
    recs = out["records"]
    t = np.array([r["setup_s"] + r["solve_s"] for r in recs]) * 1e3
    it = np.array([r["iters"] for r in recs])
    ma = np.array([r["min_alpha"] for r in recs])
    setups = sum(r["setup"] for r in recs)
    dist = np.linalg.norm(out["x"][-1, :3] - scene["ref"][-1, :3])
    say(f"   ms per control loop: mean {t.mean():.2f} max {t.max():.2f}; iterations mean {it.mean():.1f} max "
        f"{it.max()}; set-ups {setups}; min alpha over cycles {ma.min():.3f}; distance to goal {dist:.2f} m")
    assert np.all(it <= 100)
    assert np.all(np.isfinite(out["x"]))
    assert dist < 2.0
