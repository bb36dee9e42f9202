"""The synthetic receding-horizon scene (Sec. V-A shape: 32 obstacles in a
70 x 20 x 6 m corridor, a 20 x 20 x 6 m sensing window, a reference through 5
random waypoints flown in 25 s at dt = 0.1 s, horizon T = 16, sigma = 300):
checks of the generator and of the sensing and reference windows (CPU)."""
import numpy as np

import workloads


def test_scene_shape():
    sc = workloads.closed_loop_scene()
    base = sc["base"]
    assert len(sc["obstacles"]) == 32
    assert base["N"] == 16 and base["dt"] == 0.1 and base["sigma"] == 300.0
    assert sc["ref"].shape == (251, 12)
    assert np.allclose(sc["ref"][0, :3], [0, 0, 1]) and np.allclose(sc["ref"][-1, :3], [0, 70, 1])
    # the path passes through the 5 waypoints; the speed ramps up from rest
    # in 2 s, stays constant and ramps down to rest in the last 2 s
    for w in sc["waypoints"][1:-1]:
        assert np.min(np.linalg.norm(sc["ref"][:, :3] - w, axis=1)) < 0.3
    steps = np.linalg.norm(np.diff(sc["ref"][:, :3], axis=0), axis=1)
    assert np.ptp(steps[25:-25]) < 1e-3 * steps[25:-25].mean()
    assert steps[0] < 0.1 * steps[100] and steps[-1] < 0.1 * steps[100]
    speed = np.linalg.norm(sc["ref"][:, 3:6], axis=1)
    assert np.allclose(speed[1:-1], (steps[1:] + steps[:-1]) / 0.2, rtol=0.05, atol=0.05)
    for (C, d), (lo, hi) in zip(sc["obstacles"], sc["boxes"]):
        assert 6 <= len(d) <= 10
        assert -10 <= lo[0] and hi[0] <= 10 and 0 <= lo[1] and hi[1] <= 70 and lo[2] == 0 and hi[2] == 6
        # the box holds the polytope: every vertex direction's support is inside
        centre = (lo + hi) / 2
        assert np.all(C @ centre < d)


def test_sensing_window():
    sc = workloads.closed_loop_scene()
    for p in ([0.0, 20.0, 1.0], [3.0, 45.0, 2.0]):
        ids = workloads.sensed(sc, p)
        for j, (lo, hi) in enumerate(sc["boxes"]):
            inside = np.all(lo <= np.array(p) + sc["window"]) and np.all(hi >= np.array(p) - sc["window"])
            assert (j in ids) == inside
    assert len(workloads.sensed(sc, [0.0, 45.0, 1.0])) > len(workloads.sensed(sc, [0.0, 20.0, 1.0]))


def test_cycle_problem():
    sc = workloads.closed_loop_scene()
    ids = workloads.sensed(sc, [0.0, 45.0, 1.0])
    x0 = sc["ref"][150].copy()
    p = workloads.cycle_problem(sc, ids, x0, 150)
    assert p["x_ref"].shape == (1, 17, 12)
    assert np.array_equal(p["x_ref"][0], sc["ref"][150:167])
    assert int(p["obs_ptr"][-1]) == len(ids)
    q = workloads.cycle_problem(sc, ids, x0, 245)
    assert np.array_equal(q["x_ref"][0, -1], sc["ref"][-1])
