"""Seeded synthetic problem instances for the collision-avoidance ADMM path.

This module only draws geometry, dynamics models, references and costs. It
holds none of the method's arithmetic (no scale LP, no pair QP, no trajectory
QP), so both the FP64 oracle and the HIP path can consume its output.

Shapes follow the problem statement of the paper: robot = union of convex
polytope parts {x : A_i x <= b_i} posed by the state (Sec. IV-A), obstacles =
union of convex polytopes {y : C_j y <= d_j} (Sec. IV-A), dynamics
s_{t+1} = s_t + f(s_t, u_t) (Sec. IV-A, system equation) given here already
linearised about a straight reference, tracking cost with weights Q_s, Q_u
(Sec. IV-A, navigation cost).

Problem dictionary (all numpy arrays, float64 unless noted):
  dim, n_s, n_u, N (horizon), dt
  part_face_ptr int32[P+1], part_A [F_r, dim], part_b [F_r], part_off [P, dim]
  obs_ptr int32[n_scen+1]       obstacle range of each scenario
  obs_face_ptr int32[M_tot+1]   face range of each obstacle
  obs_C [F_o, dim] (unit normals), obs_d [F_o]
  A_dyn [n_s, n_s], B_dyn [n_s, n_u], c_dyn [n_s]   (one time-invariant model), or
        [n_models, ...] with dyn_ts, dyn_ss: step t of scenario s uses model
        s * dyn_ss + t * dyn_ts (optional keys, default 0)
  model, model_par   optional nonlinear model (1 bicycle, 2 quadrotor) that the
        method relinearises about every iterate; A_dyn/B_dyn/c_dyn then give the
        initial trajectory only
  pos_idx int32[dim], att_idx int32[1|3], att_kind (0 planar yaw, 1 ZYX Euler)
  Q_s [n_s, n_s], Q_u [n_u, n_u], x_ref [n_scen, N+1, n_s], x0 [n_scen, n_s]
  sigma, eps_prox, eps_pri, eps_dual
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import ConvexHull

ATT_YAW = 0
ATT_EULER_ZYX = 1

# ADMM penalty used in the paper's quadrotor experiment (Sec. V-A).
SIGMA_PAPER = 300.0


# --------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------
def box_faces(half_extents, yaw=0.0):
    """H-form of an axis-aligned box (optionally yawed about z) centred at 0."""
    h = np.asarray(half_extents, dtype=np.float64)
    d = h.size
    A = np.concatenate([np.eye(d), -np.eye(d)], axis=0)
    b = np.concatenate([h, h])
    if yaw != 0.0:
        c, s = np.cos(yaw), np.sin(yaw)
        Rz = np.eye(d)
        Rz[0, 0], Rz[0, 1], Rz[1, 0], Rz[1, 1] = c, -s, s, c
        # {x : A Rz^T x <= b} is the box rotated by Rz
        A = A @ Rz.T
    return A, b


def hull_faces(points, merge_tol=1e-9):
    """Unit-normal H-form {x : C x <= d} of the convex hull of points."""
    hull = ConvexHull(points)
    eq = hull.equations  # n.x + off <= 0 inside
    normals = eq[:, :-1]
    offs = -eq[:, -1]
    nn = np.linalg.norm(normals, axis=1)
    normals = normals / nn[:, None]
    offs = offs / nn
    keep = []
    for k in range(len(offs)):
        dup = False
        for q in keep:
            if np.linalg.norm(normals[k] - normals[q]) < merge_tol and abs(offs[k] - offs[q]) < merge_tol:
                dup = True
                break
        if not dup:
            keep.append(k)
    return normals[keep], offs[keep]


def polygon_on_circle(rng, n_faces, radius):
    """Convex polygon with n_faces vertices at sorted uniform angles on a circle."""
    while True:
        ang = np.sort(rng.uniform(0.0, 2 * np.pi, size=n_faces))
        gaps = np.diff(np.concatenate([ang, ang[:1] + 2 * np.pi]))
        if gaps.min() > 1e-3 and gaps.max() < np.pi - 1e-3:
            break
    pts = radius * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    C, d = hull_faces(pts)
    return C, d


def disc_points(rng, n, r, dim):
    """n points uniform (by volume) in a dim-ball of radius r."""
    x = rng.normal(size=(n, dim))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    rad = r * rng.uniform(size=(n, 1)) ** (1.0 / dim)
    return x * rad


# --------------------------------------------------------------------------
# dynamics models (already linearised about a straight constant-speed line)
# --------------------------------------------------------------------------
def bicycle_model(v_ref, dt=0.1, wheelbase=2.7):
    """Kinematic bicycle, state (p_x, p_y, theta, v), input (a, delta).

    Euler-discretised and linearised about theta = 0, v = v_ref, delta = 0.
    """
    A = np.eye(4)
    A[0, 3] = dt
    A[1, 2] = dt * v_ref
    B = np.zeros((4, 2))
    B[2, 1] = dt * v_ref / wheelbase
    B[3, 0] = dt
    c = np.zeros(4)
    return A, B, c


def quadrotor_model(dt=0.1, mass=1.0, J=(0.01, 0.01, 0.02), g=9.81):
    """12-state hover-linearised quadrotor (p, v, phi theta psi, omega).

    Input (dF, tau_x, tau_y, tau_z). Euler-discretised.
    """
    Ac = np.zeros((12, 12))
    Ac[0:3, 3:6] = np.eye(3)
    Ac[3, 7] = g      # v_x' = g theta
    Ac[4, 6] = -g     # v_y' = -g phi
    Ac[6:9, 9:12] = np.eye(3)
    Bc = np.zeros((12, 4))
    Bc[5, 0] = 1.0 / mass
    Bc[9, 1] = 1.0 / J[0]
    Bc[10, 2] = 1.0 / J[1]
    Bc[11, 3] = 1.0 / J[2]
    return np.eye(12) + dt * Ac, dt * Bc, np.zeros(12)


MODEL_LINEAR, MODEL_BICYCLE, MODEL_QUADROTOR = 0, 1, 2


def bicycle_step(x, u, dt=0.1, wheelbase=2.7):
    """One Euler step of the kinematic bicycle (p_x, p_y, theta, v), (a, delta)."""
    px, py, th, v = x
    a, de = u
    return np.array([px + dt * v * np.cos(th), py + dt * v * np.sin(th),
                     th + dt * v * np.tan(de) / wheelbase, v + dt * a])


def bicycle_linearised(x, u, dt=0.1, wheelbase=2.7):
    """(A, B, c) of the bicycle step linearised about (x, u):
    step(x', u') ~ A x' + B u' + c."""
    px, py, th, v = x
    a, de = u
    A = np.eye(4)
    A[0, 2] = -dt * v * np.sin(th)
    A[0, 3] = dt * np.cos(th)
    A[1, 2] = dt * v * np.cos(th)
    A[1, 3] = dt * np.sin(th)
    A[2, 3] = dt * np.tan(de) / wheelbase
    B = np.zeros((4, 2))
    B[2, 1] = dt * v / (wheelbase * np.cos(de) ** 2)
    B[3, 0] = dt
    c = bicycle_step(x, u, dt, wheelbase) - A @ x - B @ u
    return A, B, c


# --------------------------------------------------------------------------
# problem assembly
# --------------------------------------------------------------------------
def _pack_parts(parts):
    ptr = [0]
    A, b, off = [], [], []
    for (Ai, bi, oi) in parts:
        A.append(Ai)
        b.append(bi)
        off.append(oi)
        ptr.append(ptr[-1] + len(bi))
    return (np.asarray(ptr, np.int32), np.concatenate(A), np.concatenate(b),
            np.asarray(off, np.float64))


def _pack_obstacles(scen_obstacles):
    obs_ptr = [0]
    face_ptr = [0]
    C, d = [], []
    for obs in scen_obstacles:
        for (Cj, dj) in obs:
            C.append(Cj)
            d.append(dj)
            face_ptr.append(face_ptr[-1] + len(dj))
        obs_ptr.append(obs_ptr[-1] + len(obs))
    dim = C[0].shape[1] if C else 2
    return (np.asarray(obs_ptr, np.int32), np.asarray(face_ptr, np.int32),
            np.concatenate(C) if C else np.zeros((0, dim)),
            np.concatenate(d) if d else np.zeros(0))


def _straight_ref(start, direction, speed, N, dt, n_s, pos_idx, vel_idx):
    x = np.zeros((N + 1, n_s))
    for t in range(N + 1):
        x[t, pos_idx] = np.asarray(start) + np.asarray(direction) * speed * t * dt
    if vel_idx is not None:
        x[:, vel_idx] = np.asarray(direction) * speed if np.ndim(vel_idx) else speed
    return x


def _reject_near_start(center, radius, start_pts, robot_radius, margin=0.5):
    for p in start_pts:
        if np.linalg.norm(center - p) < radius + robot_radius + margin:
            return True
    return False


def _obstacles_2d_hull(rng, M, field_lo, field_hi, start_pts, robot_radius, face_range,
                       n_points=12, r=3.0):
    obs = []
    while len(obs) < M:
        c = rng.uniform(field_lo, field_hi, size=2)
        pts = disc_points(rng, n_points, r, 2)
        C, dl = hull_faces(pts)
        if not (face_range[0] <= len(dl) <= face_range[1]):
            continue
        rad = np.linalg.norm(pts, axis=1).max()
        if _reject_near_start(c, rad, start_pts, robot_radius):
            continue
        obs.append((C, dl + C @ c))
    return obs


def _finish(prob):
    prob.setdefault("eps_pri", 1e-4)
    prob.setdefault("eps_dual", 1e-4)
    prob.setdefault("eps_prox", 1e-1)
    return prob


def config_c1(seed=16):
    """2D: one 4.5 x 2 m rectangle, 3 hull obstacles (4-8 faces) in a 40 x 40 m
    field, bicycle at 20 m/s, N = 20, sigma = 1."""
    rng = np.random.default_rng(seed)
    N, dt, v = 20, 0.1, 20.0
    A_r, b_r = box_faces([2.25, 1.0])
    parts = [(A_r, b_r, np.zeros(2))]
    start = np.array([0.0, 20.0])
    start_pts = [start, start + np.array([v * dt, 0.0])]
    obs = _obstacles_2d_hull(rng, 3, 0.0, 40.0, start_pts, np.hypot(2.25, 1.0), (4, 8))
    return _assemble_2d(parts, [obs], N, dt, v, start[None, :], sigma=1.0)


def config_c2(seed=10):
    """2D: cab 3 x 2.5 + trailer 9 x 2.5 (rigid), 40 hull obstacles (3-10 faces)
    in a 100 x 100 m field, bicycle at 20 m/s, N = 50 -> 4000 pairs, sigma as
    in the paper's experiment."""
    rng = np.random.default_rng(seed)
    N, dt, v = 50, 0.1, 20.0
    A_c, b_c = box_faces([1.5, 1.25])
    A_t, b_t = box_faces([4.5, 1.25])
    parts = [(A_c, b_c, np.array([4.5, 0.0])), (A_t, b_t, np.array([-1.5, 0.0]))]
    start = np.array([0.0, 50.0])
    start_pts = [start, start + np.array([v * dt, 0.0])]
    obs = _obstacles_2d_hull(rng, 40, 0.0, 100.0, start_pts, np.hypot(6.0, 1.25), (3, 10))
    return _assemble_2d(parts, [obs], N, dt, v, start[None, :], sigma=SIGMA_PAPER)


def config_c2tv(seed=13, n_scen=4, N=50, M=10, v=12.0, steer=(-0.05, -0.02, 0.02, 0.05)):
    """2D, time-varying models: n_scen scenarios of the C1 rectangle, each
    following its own arc (constant steering angle, 12 m/s) with the bicycle
    linearised about every step of its reference (one model per scenario and
    step: dyn_ss = N, dyn_ts = 1); M hull obstacles (3-10 faces, 2 m discs)
    centred 2.5-5 m to either side of the arc."""
    rng = np.random.default_rng(seed)
    dt, L = 0.1, 2.7
    A_r, b_r = box_faces([2.25, 1.0])
    parts = [(A_r, b_r, np.zeros(2))]
    x_ref = np.zeros((n_scen, N + 1, 4))
    Ad = np.zeros((n_scen * N, 4, 4))
    Bd = np.zeros((n_scen * N, 4, 2))
    cd = np.zeros((n_scen * N, 4))
    scen = []
    for s in range(n_scen):
        de = steer[s % len(steer)]
        x = np.array([0.0, 20.0, 0.0, v])
        x_ref[s, 0] = x
        for t in range(N):
            Ad[s * N + t], Bd[s * N + t], cd[s * N + t] = bicycle_linearised(x, (0.0, de), dt, L)
            x = bicycle_step(x, (0.0, de), dt, L)
            x_ref[s, t + 1] = x
        start_pts = [x_ref[s, 0, :2], x_ref[s, 1, :2], x_ref[s, 2, :2]]
        obs = []
        while len(obs) < M:
            t = int(rng.integers(10, N + 1))
            th = x_ref[s, t, 2]
            nrm = np.array([-np.sin(th), np.cos(th)])
            c = x_ref[s, t, :2] + rng.choice([-1.0, 1.0]) * rng.uniform(2.5, 5.0) * nrm
            pts = disc_points(rng, 12, 2.0, 2)
            C, dl = hull_faces(pts)
            if not (3 <= len(dl) <= 10):
                continue
            rad = np.linalg.norm(pts, axis=1).max()
            if _reject_near_start(c, rad, start_pts, np.hypot(2.25, 1.0)):
                continue
            obs.append((C, dl + C @ c))
        scen.append(obs)
    ptr, A, b, off = _pack_parts(parts)
    obs_ptr, face_ptr, C, d = _pack_obstacles(scen)
    return _finish(dict(
        dim=2, n_s=4, n_u=2, N=N, dt=dt,
        part_face_ptr=ptr, part_A=A, part_b=b, part_off=off,
        obs_ptr=obs_ptr, obs_face_ptr=face_ptr, obs_C=C, obs_d=d,
        A_dyn=Ad, B_dyn=Bd, c_dyn=cd, dyn_ts=1, dyn_ss=N,
        pos_idx=np.array([0, 1], np.int32), att_idx=np.array([2], np.int32), att_kind=ATT_YAW,
        Q_s=np.diag([1.0, 1.0, 0.1, 0.1]), Q_u=np.diag([0.1, 0.1]),
        x_ref=x_ref, x0=x_ref[:, 0, :].copy(), sigma=SIGMA_PAPER))


def config_c2sqp(seed=10):
    """C2 with the nonlinear kinematic bicycle relinearised about every
    iterate (the given straight-line linearisation sets the initial
    trajectory only)."""
    p = config_c2(seed)
    p.update(model=MODEL_BICYCLE, model_par=np.array([p["dt"], 2.7]))
    return p


def config_c2b(seed=10, v_range=(19.9, 20.3), a_range=(-3.0, 1.0), steer=0.07):
    """C2 with state and input bounds: speed in v_range, acceleration in
    a_range, steering within +-steer (the other states free). The bounds cut
    what the unbounded C2 solve reaches (speed 19.95-21.7 m/s, acceleration
    up to 2 m/s^2, steering up to 0.11 rad), so some stay active at the
    solution."""
    p = config_c2(seed)
    inf = np.inf
    p.update(s_min=np.array([-inf, -inf, -inf, v_range[0]]), s_max=np.array([inf, inf, inf, v_range[1]]),
             u_min=np.array([a_range[0], -steer]), u_max=np.array([a_range[1], steer]))
    return p


def closed_loop_scene(seed=41, n_sparse=8, n_dense=24, N=16, duration=25.0, dt=0.1, sigma=SIGMA_PAPER,
                      path_clearance=0.0):
    """The receding-horizon workload of Sec. V-A, synthetic (the AirSim scene is
    not available): a 70 x 20 x 6 m corridor (x in [-10, 10], y in [0, 70],
    z in [0, 6]) with 32 obstacles, n_sparse in an obstacle-sparse stretch
    (y in [8, 32]) and n_dense in an obstacle-dense one (y in [36, 64]); each a
    vertical prism over the full height (a regular polygon of U{4..8} sides,
    circumradius U(0.4, 1.0) m, random yaw; centres at least 2.4 m apart, 3 m
    from the start and goal, and the circumradius + path_clearance from the
    reference path, so that no obstacle blocks it head-on but those beside it
    still reach into the robot's swept width). The quadrotor as one box of
    0.8 x 0.8 x 0.2 m (its frame with the rotors), the nonlinear model
    relinearised every iteration, horizon N = 16, dt = 0.1 s, sigma = 300, the
    C3 weights scaled by 100 (the tracking cost against the penalty), the
    corridor's walls, floor and ceiling as state bounds on the position. Reference: a Catmull-Rom curve from (0, 0, 1) through 5
    random waypoints (y = 70 k / 6, x ~ U(-6, 6), z ~ U(0.8, 2.5)) to
    (0, 70, 1), flown in `duration` seconds with a trapezoidal speed profile
    (2 s to speed up from rest and 2 s to stop), sampled every dt, with the
    path's velocity and zero attitude and rates.
    Returns the scene: base problem fields, obstacles as (C, d) and their
    bounding boxes, the sampled reference ref[K + 1, 12] and the start state."""
    rng = np.random.default_rng(seed)
    A_b, b_b = box_faces([0.4, 0.4, 0.1])
    parts = [(A_b, b_b, np.zeros(3))]
    start, goal = np.array([0.0, 0.0, 1.0]), np.array([0.0, 70.0, 1.0])
    way = [start]
    for k in range(1, 6):
        way.append(np.array([rng.uniform(-6.0, 6.0), 70.0 * k / 6.0, rng.uniform(0.8, 2.5)]))
    way.append(goal)
    way = np.array(way)
    # the curve, densely sampled (uniform Catmull-Rom, end points doubled)
    P4 = np.concatenate([way[:1], way, way[-1:]])
    dense = []
    for i in range(len(way) - 1):
        p0, p1, p2, p3 = P4[i], P4[i + 1], P4[i + 2], P4[i + 3]
        for tt in np.linspace(0.0, 1.0, 400, endpoint=False):
            dense.append(0.5 * (2 * p1 + (p2 - p0) * tt + (2 * p0 - 5 * p1 + 4 * p2 - p3) * tt ** 2
                                + (3 * p1 - p0 - 3 * p2 + p3) * tt ** 3))
    dense.append(way[-1])
    dense = np.array(dense)
    obstacles, boxes, centres = [], [], []
    for n, (ylo, yhi) in ((n_sparse, (8.0, 32.0)), (n_dense, (36.0, 64.0))):
        placed = 0
        while placed < n:
            c = np.array([rng.uniform(-8.0, 8.0), rng.uniform(ylo, yhi), 3.0])
            if any(np.hypot(*(c[:2] - q[:2])) < 2.4 for q in centres):
                continue
            if min(np.hypot(*(c[:2] - start[:2])), np.hypot(*(c[:2] - goal[:2]))) < 3.0:
                continue
            sides = int(rng.integers(4, 9))
            rad = rng.uniform(0.4, 1.0)
            # no obstacle blocks the path head-on: its centre keeps rad + 0.2 m
            # from the path (the robot's arms reach 0.45 m, so it still has to
            # swerve around the obstacles that graze the path)
            if np.min(np.hypot(dense[:, 0] - c[0], dense[:, 1] - c[1])) < rad + path_clearance:
                continue
            yaw = rng.uniform(0.0, 2.0 * np.pi)
            R = np.array([[np.cos(yaw), -np.sin(yaw), 0.0], [np.sin(yaw), np.cos(yaw), 0.0], [0.0, 0.0, 1.0]])
            C, dl = prism_faces(sides, rad, 3.0, R)
            obstacles.append((C, dl + C @ c))
            boxes.append((c - np.array([rad, rad, 3.0]), c + np.array([rad, rad, 3.0])))
            centres.append(c)
            placed += 1
    arc = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(dense, axis=0), axis=1))])
    K = int(round(duration / dt))
    ramp = 2.0
    vmax = arc[-1] / (duration - ramp)

    def s_of(t):   # arc length flown at time t
        if t <= ramp:
            return 0.5 * vmax * t * t / ramp
        if t >= duration - ramp:
            r = duration - t
            return arc[-1] - 0.5 * vmax * r * r / ramp
        return vmax * (t - 0.5 * ramp)

    ref = np.zeros((K + 1, 12))
    for k in range(K + 1):
        t = k * dt
        a = min(max(s_of(t), 0.0), arc[-1])
        i = min(int(np.searchsorted(arc, a, side="right")) - 1, len(dense) - 2)
        seg = arc[i + 1] - arc[i]
        tdir = (dense[i + 1] - dense[i]) / seg
        ref[k, :3] = dense[i] + (a - arc[i]) * tdir
        speed = (s_of(min(t + 1e-3, duration)) - s_of(max(t - 1e-3, 0.0))) / (min(t + 1e-3, duration) - max(t - 1e-3, 0.0))
        ref[k, 3:6] = speed * tdir
    ptr, A, b, off = _pack_parts(parts)
    Ad, Bd, cd = quadrotor_model(dt)
    base = dict(dim=3, n_s=12, n_u=4, N=N, dt=dt,
                part_face_ptr=ptr, part_A=A, part_b=b, part_off=off,
                A_dyn=Ad, B_dyn=Bd, c_dyn=cd,
                pos_idx=np.array([0, 1, 2], np.int32), att_idx=np.array([6, 7, 8], np.int32),
                att_kind=ATT_EULER_ZYX,
                Q_s=100.0 * np.diag([1, 1, 1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.01, 0.01, 0.01]),
                Q_u=100.0 * np.diag([0.1, 1.0, 1.0, 1.0]), sigma=sigma,
                model=MODEL_QUADROTOR, model_par=np.array([dt, 1.0, 0.01, 0.01, 0.02, 9.81]),
                # the corridor as state bounds (Sec. IV-A eq. MPC_opt_origin): the
                # robot's centre stays 0.5 m inside its walls, floor and ceiling
                s_min=np.array([-9.5, -np.inf, 0.5] + [-np.inf] * 9),
                s_max=np.array([9.5, np.inf, 5.5] + [np.inf] * 9))
    x_start = np.zeros(12)
    x_start[:3] = start
    return dict(base=_finish(base), obstacles=obstacles, boxes=boxes, ref=ref, x_start=x_start,
                waypoints=way, window=np.array([10.0, 10.0, 3.0]))


def sensed(scene, position):
    """Indices of the obstacles the robot senses at `position`: those whose
    bounding box meets the 20 x 20 x 6 m window centred on it (Sec. V-A)."""
    w = scene["window"]
    lo, hi = np.asarray(position) - w, np.asarray(position) + w
    return [j for j, (blo, bhi) in enumerate(scene["boxes"]) if np.all(blo <= hi) and np.all(bhi >= lo)]


def reference_window(scene, k):
    """x_ref for cycle k: the reference samples k .. k + N (held at the end)."""
    ref = scene["ref"]
    N = scene["base"]["N"]
    idx = np.minimum(np.arange(k, k + N + 1), len(ref) - 1)
    return ref[idx][None]


def cycle_problem(scene, ids, x0, k):
    """The problem of cycle k: the sensed obstacles ids, the measured state x0
    and the reference window of cycle k (one scenario)."""
    p = dict(scene["base"])
    p = with_obstacles(p, [[scene["obstacles"][j] for j in ids]])
    p["x_ref"] = reference_window(scene, k)
    p["x0"] = np.asarray(x0, np.float64)[None].copy()
    return p


def config_c3sqp(seed=25):
    """C3 with the nonlinear quadrotor relinearised about every iterate."""
    p = config_c3(seed)
    p.update(model=MODEL_QUADROTOR, model_par=np.array([p["dt"], 1.0, 0.01, 0.01, 0.02, 9.81]))
    return p


def config_c4(seed=101, n_scen=256, m_range=(10, 80), f_range=(3, 12)):
    """Batched 2D: n_scen scenarios of the C1 robot/model, obstacle counts
    uniform in m_range, polygon faces uniform in f_range, 8 m/s, N = 50."""
    N, dt, v = 50, 0.1, 8.0
    A_r, b_r = box_faces([2.25, 1.0])
    parts = [(A_r, b_r, np.zeros(2))]
    scen = []
    starts = []
    for s in range(n_scen):
        rng = np.random.default_rng(seed + s)
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        start = np.array([0.0, 20.0])
        start_pts = [start, start + np.array([v * dt, 0.0]), start + np.array([2 * v * dt, 0.0])]
        obs = []
        while len(obs) < M:
            F = int(rng.integers(f_range[0], f_range[1] + 1))
            rad = rng.uniform(0.5, 3.0)
            c = rng.uniform(0.0, 40.0, size=2)
            if _reject_near_start(c, rad, start_pts, np.hypot(2.25, 1.0)):
                continue
            C, dl = polygon_on_circle(rng, F, rad)
            obs.append((C, dl + C @ c))
        scen.append(obs)
        starts.append(start)
    return _assemble_2d(parts, scen, N, dt, v, np.asarray(starts), sigma=1.0)


def pair_batch_c4_shape(n_pairs, seed=7):
    """A stateless batch of dual-update QP inputs of the batched 2D shape, for
    streaming the stateless pair-QP entry point: per pair the 4.5 x 2 m
    rectangle's 4 rows (0, a_k) with kappa = b, F ~ U{3..12} obstacle rows
    (d', c) with unit normals at uniform angles and clearances
    d' ~ U(-0.5, 6) m, and the row (1, 0); yhat >= 0 exponential, bhat near
    (1, 0, 0). Returns row_ptr int32 [P+1], K [rows, 3], kappa, yhat [rows],
    bhat [P, 3] (float32)."""
    rng = np.random.default_rng(seed)
    A_r, b_r = box_faces([2.25, 1.0])
    F = rng.integers(3, 13, size=n_pairs)
    n = 4 + F + 1
    row_ptr = np.zeros(n_pairs + 1, np.int64)
    np.cumsum(n, out=row_ptr[1:])
    rows = int(row_ptr[-1])
    K = np.zeros((rows, 3), np.float32)
    kap = np.zeros(rows, np.float32)
    start = row_ptr[:-1]
    for k in range(4):
        K[start + k, 1:] = A_r[k]
        kap[start + k] = b_r[k]
    # obstacle rows: row index start + 4 + j for j < F
    pair_of_row = np.repeat(np.arange(n_pairs), n)
    local = np.arange(rows) - start[pair_of_row]
    obs_rows = np.nonzero((local >= 4) & (local < n[pair_of_row] - 1))[0]
    ang = rng.uniform(0.0, 2 * np.pi, size=obs_rows.size)
    K[obs_rows, 0] = rng.uniform(-0.5, 6.0, size=obs_rows.size)
    K[obs_rows, 1] = np.cos(ang)
    K[obs_rows, 2] = np.sin(ang)
    K[row_ptr[1:] - 1, 0] = 1.0
    yhat = rng.exponential(0.1, size=rows).astype(np.float32)
    bhat = np.zeros((n_pairs, 3), np.float32)
    bhat[:, 0] = 1.0 + rng.normal(0.0, 0.1, size=n_pairs)
    bhat[:, 1:] = rng.normal(0.0, 0.1, size=(n_pairs, 2))
    return row_ptr.astype(np.int32), K, kap, yhat, bhat


def _assemble_2d(parts, scen_obstacles, N, dt, v, starts, sigma):
    ptr, A, b, off = _pack_parts(parts)
    obs_ptr, face_ptr, C, d = _pack_obstacles(scen_obstacles)
    Ad, Bd, cd = bicycle_model(v, dt)
    n_scen = len(scen_obstacles)
    x_ref = np.zeros((n_scen, N + 1, 4))
    for s in range(n_scen):
        x_ref[s] = _straight_ref(starts[s], [1.0, 0.0], v, N, dt, 4, [0, 1], None)
        x_ref[s, :, 3] = v
    return _finish(dict(
        dim=2, n_s=4, n_u=2, N=N, dt=dt,
        part_face_ptr=ptr, part_A=A, part_b=b, part_off=off,
        obs_ptr=obs_ptr, obs_face_ptr=face_ptr, obs_C=C, obs_d=d,
        A_dyn=Ad, B_dyn=Bd, c_dyn=cd,
        pos_idx=np.array([0, 1], np.int32), att_idx=np.array([2], np.int32), att_kind=ATT_YAW,
        Q_s=np.diag([1.0, 1.0, 0.1, 0.1]), Q_u=np.diag([0.1, 0.1]),
        x_ref=x_ref, x0=x_ref[:, 0, :].copy(), sigma=sigma))


def config_c3(seed=25, M=200, N=40, k_range=(7, 12)):
    """3D: quadrotor = body box + two crossed arm boxes, M hull polyhedra
    (hulls of k ~ U{7..12} points in a 1.5 m ball), 50^3 m box, 12.5 m/s, N = 40."""
    rng = np.random.default_rng(seed)
    dt, v = 0.1, 12.5
    A_b, b_b = box_faces([0.15, 0.15, 0.05])
    A_1, b_1 = box_faces([0.4, 0.03, 0.02], yaw=np.pi / 4)
    A_2, b_2 = box_faces([0.4, 0.03, 0.02], yaw=-np.pi / 4)
    parts = [(A_b, b_b, np.zeros(3)), (A_1, b_1, np.zeros(3)), (A_2, b_2, np.zeros(3))]
    start = np.array([0.0, 25.0, 25.0])
    start_pts = [start, start + np.array([v * dt, 0, 0])]
    obs = []
    while len(obs) < M:
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        pts = disc_points(rng, k, 1.5, 3)
        try:
            C, dl = hull_faces(pts)
        except Exception:
            continue
        if not (6 <= len(dl) <= 20):
            continue
        c = rng.uniform(0.0, 50.0, size=3)
        rad = np.linalg.norm(pts, axis=1).max()
        if _reject_near_start(c, rad, start_pts, 0.45):
            continue
        obs.append((C, dl + C @ c))
    ptr, A, b, off = _pack_parts(parts)
    obs_ptr, face_ptr, C, d = _pack_obstacles([obs])
    Ad, Bd, cd = quadrotor_model(dt)
    x_ref = np.zeros((1, N + 1, 12))
    x_ref[0] = _straight_ref(start, [1.0, 0.0, 0.0], v, N, dt, 12, [0, 1, 2], None)
    x_ref[0, :, 3] = v
    return _finish(dict(
        dim=3, n_s=12, n_u=4, N=N, dt=dt,
        part_face_ptr=ptr, part_A=A, part_b=b, part_off=off,
        obs_ptr=obs_ptr, obs_face_ptr=face_ptr, obs_C=C, obs_d=d,
        A_dyn=Ad, B_dyn=Bd, c_dyn=cd,
        pos_idx=np.array([0, 1, 2], np.int32), att_idx=np.array([6, 7, 8], np.int32),
        att_kind=ATT_EULER_ZYX,
        Q_s=np.diag([1, 1, 1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.01, 0.01, 0.01]).astype(np.float64),
        Q_u=np.diag([0.1, 1.0, 1.0, 1.0]),
        x_ref=x_ref, x0=x_ref[:, 0, :].copy(), sigma=SIGMA_PAPER))


def regular_polygon_faces(n_faces, radius):
    """Faces (A, b) of a regular polygon with n_faces edges whose vertices lie
    on a circle of the given radius, centred at the origin (b > 0)."""
    ang = 2.0 * np.pi * (np.arange(n_faces) + 0.5) / n_faces
    A = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    b = np.full(n_faces, radius * np.cos(np.pi / n_faces))
    return A, b


def config_edge_2d(seed=3, N=20, M=4, f_range=(17, 32), part_faces=8, sigma=SIGMA_PAPER):
    """Edge sizes in 2D: one robot part with part_faces faces (a regular
    polygon of radius 2 m), M polygon obstacles with F ~ U{f_range} faces on
    circles of radius U(1, 2.5) m placed along the first 2/3 of the path with
    lateral offsets of 2.5-4.5 m (so that pairs become active), bicycle at
    10 m/s, horizon N."""
    rng = np.random.default_rng(seed)
    dt, v = 0.1, 10.0
    A_r, b_r = regular_polygon_faces(part_faces, 2.0)
    parts = [(A_r, b_r, np.zeros(2))]
    start = np.array([0.0, 20.0])
    start_pts = [start, start + np.array([v * dt, 0.0])]
    length = max(v * dt * N * 2.0 / 3.0, 8.0)
    obs = []
    while len(obs) < M:
        F = int(rng.integers(f_range[0], f_range[1] + 1))
        rad = rng.uniform(1.0, 2.5)
        c = start + np.array([rng.uniform(4.0, 4.0 + length), rng.choice([-1.0, 1.0]) * rng.uniform(2.5, 4.5)])
        if _reject_near_start(c, rad, start_pts, 2.0):
            continue
        C, dl = polygon_on_circle(rng, F, rad)
        obs.append((C, dl + C @ c))
    return _assemble_2d(parts, [obs], N, dt, v, start[None, :], sigma=sigma)


def prism_faces(n_sides, radius, half_height, R):
    """Faces (A, b) of a regular n_sides-gon prism (circumradius radius,
    height 2 half_height) rotated by R, centred at the origin: n_sides + 2
    faces, b > 0."""
    ang = 2.0 * np.pi * (np.arange(n_sides) + 0.5) / n_sides
    side = np.stack([np.cos(ang), np.sin(ang), np.zeros(n_sides)], axis=1)
    A = np.concatenate([side, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]]) @ R.T
    b = np.concatenate([np.full(n_sides, radius * np.cos(np.pi / n_sides)), [half_height, half_height]])
    return A, b


def random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def config_edge_3d(seed=5, N=10, M=6, side_range=(23, 30), sigma=SIGMA_PAPER):
    """Edge sizes in 3D: the C3 quadrotor and model, M randomly rotated
    regular prisms with n ~ U{side_range} sides (n + 2 = 25..32 faces,
    circumradius U(0.6, 1.5) m, half height U(0.4, 1.2) m) along the path,
    their centres 0-0.6 m beyond their bounding radius from it, horizon N."""
    rng = np.random.default_rng(seed)
    dt, v = 0.1, 12.5
    base = config_c3(seed=25, M=1, N=N)
    start = np.array([0.0, 25.0, 25.0])
    start_pts = [start, start + np.array([v * dt, 0, 0])]
    length = max(v * dt * N * 2.0 / 3.0, 4.0)
    obs = []
    while len(obs) < M:
        n = int(rng.integers(side_range[0], side_range[1] + 1))
        rad, hh = rng.uniform(0.6, 1.5), rng.uniform(0.4, 1.2)
        C, dl = prism_faces(n, rad, hh, random_rotation(rng))
        u = rng.standard_normal(2)
        u /= np.linalg.norm(u)
        c = start + np.array([rng.uniform(3.0, 3.0 + length), 0.0, 0.0])
        c[1:] += u * (np.hypot(rad, hh) + rng.uniform(0.0, 0.6))
        if _reject_near_start(c, np.hypot(rad, hh), start_pts, 0.45):
            continue
        obs.append((C, dl + C @ c))
    out = with_obstacles(base, [obs])
    out["sigma"] = sigma
    return out


CONFIGS = {
    "c1": config_c1,
    "c2": config_c2,
    "c3": config_c3,
    "c4": config_c4,
    "c2tv": config_c2tv,
    "c2sqp": config_c2sqp,
    "c2b": config_c2b,
    "c3sqp": config_c3sqp,
}


def make(name, **kw):
    return CONFIGS[name](**kw)


def select_scenarios(prob, idx):
    """Sub-problem holding only the scenarios listed in idx (same robot/model)."""
    out = dict(prob)
    obs_ptr = prob["obs_ptr"]
    fptr = prob["obs_face_ptr"]
    new_obs_ptr = [0]
    new_fptr = [0]
    C, d = [], []
    for s in idx:
        for j in range(obs_ptr[s], obs_ptr[s + 1]):
            C.append(prob["obs_C"][fptr[j]:fptr[j + 1]])
            d.append(prob["obs_d"][fptr[j]:fptr[j + 1]])
            new_fptr.append(new_fptr[-1] + fptr[j + 1] - fptr[j])
        new_obs_ptr.append(new_obs_ptr[-1] + obs_ptr[s + 1] - obs_ptr[s])
    dim = prob["dim"]
    out["obs_ptr"] = np.asarray(new_obs_ptr, np.int32)
    out["obs_face_ptr"] = np.asarray(new_fptr, np.int32)
    out["obs_C"] = np.concatenate(C) if C else np.zeros((0, dim))
    out["obs_d"] = np.concatenate(d) if d else np.zeros(0)
    out["x_ref"] = prob["x_ref"][list(idx)].copy()
    out["x0"] = prob["x0"][list(idx)].copy()
    ss = int(prob.get("dyn_ss", 0))
    if ss:
        # per-scenario models: the models of the kept scenarios, in order
        ts, N = int(prob.get("dyn_ts", 0)), prob["N"]
        span = (N - 1) * ts + 1
        sel = np.concatenate([np.arange(s * ss, s * ss + span) for s in idx])
        for k in ("A_dyn", "B_dyn", "c_dyn"):
            out[k] = np.asarray(prob[k])[sel].copy()
        out["dyn_ss"] = span
    return out


def with_obstacles(prob, scen_obstacles):
    """Copy of prob with the obstacle lists replaced (one list per scenario)."""
    out = dict(prob)
    obs_ptr, face_ptr, C, d = _pack_obstacles(scen_obstacles)
    if C.shape[0] == 0:
        C = np.zeros((0, prob["dim"]))
    out.update(obs_ptr=obs_ptr, obs_face_ptr=face_ptr, obs_C=C, obs_d=d)
    return out


def n_scenarios(prob):
    return len(prob["obs_ptr"]) - 1


def block_layout(prob):
    """Canonical pair-block enumeration shared by both sides of the boundary.

    Block b enumerates (scenario s, robot part i, obstacle j) in that nesting
    order; it holds the N pairs t = 1..N. Block b has n_b = n_r,i + n_o,j + 1
    dual rows (lambda, mu, gamma). Returns arrays (scen, part, obs, n_rows,
    y_off) with y_off in floats (rows x N per block).
    """
    N = prob["N"]
    P = len(prob["part_face_ptr"]) - 1
    pf = prob["part_face_ptr"]
    of = prob["obs_face_ptr"]
    op = prob["obs_ptr"]
    scen, part, obs, nrow, yoff = [], [], [], [], []
    off = 0
    for s in range(len(op) - 1):
        for i in range(P):
            for j in range(op[s], op[s + 1]):
                n = (pf[i + 1] - pf[i]) + (of[j + 1] - of[j]) + 1
                scen.append(s)
                part.append(i)
                obs.append(j)
                nrow.append(n)
                yoff.append(off)
                off += n * N
    return (np.asarray(scen, np.int64), np.asarray(part, np.int64), np.asarray(obs, np.int64),
            np.asarray(nrow, np.int64), np.asarray(yoff, np.int64), off)
