#!/usr/bin/env python3
"""Benchmark of the ADMM collision-avoidance hot path on one MI355X.

Headline (top level): the batched workload, 256 independent 2D scenarios
(obstacle counts U{10..80}, faces U{3..12}, N = 50, about 560k pair QPs per
iteration) in one handle. A step is one batched solve with inputs resident in
HBM: reset to the initial iterate (obstacle-free LQ trajectory, scale-LP
certificates), 50 ADMM iterations by HIP-graph replay (pair QPs, trajectory
QP, multiplier update, residual test; scenarios whose stopping test holds are
skipped from then on) and the final scale certificate. `value` counts the pair
QPs actually solved (sum over scenarios of pairs x iterations run) per second.

Beside it: the batched-vs-plain comparison (the same 256 scenarios as 256
separate handles on one stream), the pair kernel's HBM roofline figure (HIP
events on the handle's stream), the single-scenario legs C2 (2D, solved to the
1e-4 residuals) and C3 (3D), the stateless pair-QP entry point streamed over
2^22 pairs, the reverse pass (backward/forward), and the FP64 oracle on the
host cores over the same batched workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs ...]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
_CSRC = "paper_2406_07048_amd/csrc/"
_COMMON = (_CSRC + "cadmm_solvers.h", _CSRC + "cadmm_device.h", _CSRC + "cadmm_internal.h")
# the sources each profiled kernel is built from (a committed counter summary
# counts only while they are unchanged)
KERNEL_SOURCES = {
    "pair_phase_kernel": (_CSRC + "cadmm_kernels.hip",) + _COMMON,
    "pair_qp_batch_kernel": (_CSRC + "cadmm_batch.hip",) + _COMMON,
}
METRIC = "pair-QP solves/sec & ADMM iters/sec at res 1e-4 (batched vs plain); backward/forward ratio"

WORKLOADS = {
    "c4": dict(desc="256 2D scenarios (4.5x2 m rectangle, bicycle at 8 m/s), obstacles U{10..80} with "
                    "U{3..12} faces in a 40x40 m field, N=50, sigma=1, 50 ADMM iterations", iters=50),
    "c2": dict(desc="2D cab+trailer (2 parts x 4 faces), 40 hull obstacles (3-10 faces), N=50, "
                    "4000 pair QPs/iteration, up to 200 ADMM iterations, sigma=300", iters=200),
    "c3": dict(desc="3D quadrotor (3 boxes), 200 hull polyhedra (6-20 faces), N=40, "
                    "24000 pair QPs/iteration, up to 200 ADMM iterations, sigma=300", iters=200),
    "c1": dict(desc="2D rectangle, 3 obstacles, N=20, 60 pair QPs/iteration, 50 ADMM iterations", iters=50),
    "c2tv": dict(desc="4 2D scenarios on curved references with one linearised bicycle model per scenario and "
                      "step, 10 hull obstacles each, N=50, up to 200 ADMM iterations, sigma=300", iters=200),
    "c2sqp": dict(desc="the C2 problem with the nonlinear kinematic bicycle relinearised about every iterate "
                       "(one SQP step per ADMM iteration), up to 200 iterations", iters=200),
    "c3sqp": dict(desc="the C3 problem with the nonlinear quadrotor relinearised about every iterate, "
                       "up to 200 iterations", iters=200),
    "c2b": dict(desc="the C2 problem with speed, acceleration and steering bounds (bounded trajectory QP every "
                     "iteration), up to 200 iterations", iters=200),
}
ALL_LEGS = ("c4", "plain", "c2", "c3", "c2tv", "c2sqp", "c3sqp", "c2b", "stream", "stream2", "lemke", "loop", "grad",
            "cpu")
VALU_PEAK_INSTS = 256 * 2.4e9   # wave-wide VALU instructions per second: 256 CUs x 2.4 GHz x one per CU clock


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pair_bytes(prob):
    """Algorithmic HBM bytes of one pair-phase launch, the per-pair figure of
    the method's hot path: every pair reads its previous duals and writes the
    new ones (2 n floats) and reads and writes its multipliers (2 (dim + 1)
    floats, the update of Sec. IV-B counted with the pair that owns them);
    every obstacle face (normal and offset, dim + 1 floats) is read once. The
    trajectory is a few KB per scenario."""
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
    N, dim = prob["N"], prob["dim"]
    return 4.0 * (2 * tot + 2 * len(sc) * N * (1 + dim)) + 4.0 * len(prob["obs_d"]) * (dim + 1)


def partial_bytes(n_wg, prob):
    """Bytes of per-workgroup contribution sums the pair kernel writes beside
    the algorithmic traffic (nc floats for each of the N steps)."""
    nq = prob["dim"] + (1 if prob["dim"] == 2 else 3)
    return 4.0 * n_wg * (nq * (nq + 1) // 2 + nq) * prob["N"]


def pairs_per_scenario(prob):
    sc = workloads.block_layout(prob)[0]
    return np.bincount(sc, minlength=workloads.n_scenarios(prob)) * prob["N"]


def kernel_source_hash(kernel="pair_phase_kernel"):
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _summary(name, suffix, kernel, launch):
    """Key-value lines of profiles/<name>_<suffix>.txt when it was taken from
    the current sources of `kernel` (and, given, at the launch shape)."""
    path = os.path.join(ROOT, "profiles", f"{name}_{suffix}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash(kernel):
        return None
    if launch is not None and kv.get("launch") != f"{launch[0]},{launch[1]}":
        return None
    return kv


def measured_traffic(name, launch=None, kernel="pair_phase_kernel"):
    """HBM bytes per launch of a kernel from the committed counter summary
    profiles/<name>_hbm_traffic.txt (FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by what the same counters read for a plain copy of known size).
    None when the summary is missing, was taken from other kernel sources or,
    given launch = (blocks per workgroup, lanes per pair), at another launch
    shape."""
    kv = _summary(name, "hbm_traffic", kernel, launch)
    return None if kv is None else float(kv["traffic_bytes_per_launch"])


def measured_valu(name, launch=None, kernel="pair_phase_kernel"):
    """VALU instructions per launch of a kernel from the committed counter
    summary profiles/<name>_valu.txt (SQ_INSTS_VALU per dispatch, with the
    busy counters beside it); None when missing, taken from other sources or
    at another launch shape."""
    kv = _summary(name, "valu", kernel, launch)
    return None if kv is None else float(kv["valu_insts_per_dispatch"])


def valu_rate(insts, ms):
    """Wave-wide VALU instructions issued per second against the issue peak
    (one per CU per clock), from counted instructions and the live duration."""
    if insts is None:
        return None
    rate = insts / (ms * 1e-3)
    return {"insts_per_launch": insts, "issue_rate": rate, "peak": VALU_PEAK_INSTS, "frac": rate / VALU_PEAK_INSTS}


def roofline(bytes_launch, ms, traffic, kernel, **extra):
    gbs = bytes_launch / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "traffic": traffic, "kernel": kernel, "bytes_per_launch": bytes_launch, "ms_per_launch": ms}
    out.update(extra)
    return out


def time_solves(h, iters, steps, torch):
    """Mean seconds of reset + iters iterations (graph replay) + the final
    scale certificate, with no host synchronisation inside a step."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.reset()
        h.iterate(iters)
        h.scales()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def make_handle(cadmm, prob, shape):
    if shape:
        w, g = (int(v) for v in shape.split(","))
        return cadmm.Handle(prob, waves_per_group=w, lanes_per_pair=g)
    return cadmm.Handle(prob)


def residual_summary(prob, res, rp, rd):
    """Per-scenario residuals after the timed solve, and the first iteration
    at which the literal stopping test (Sec. IV-B, 1e-4) held."""
    first = []
    for s in range(rp.shape[1]):
        ok = np.nonzero((rp[:, s] <= prob["eps_pri"]) & (rd[:, s] <= prob["eps_dual"]))[0]
        first.append(int(ok[0]) + 1 if ok.size else None)
    conv = [r["converged"] for r in res]
    out = {"scenarios": len(res), "converged_at_1e-4": int(sum(conv)),
           "r_pri_median": float(np.median([r["r_pri"] for r in res])),
           "r_dual_median": float(np.median([r["r_dual"] for r in res])),
           "min_alpha_min": float(min(r["min_alpha"] for r in res))}
    if len(res) == 1:
        out.update({"r_pri": res[0]["r_pri"], "r_dual": res[0]["r_dual"], "first_iter_at_1e-4": first[0],
                    "cost": res[0]["cost"], "min_alpha": res[0]["min_alpha"]})
    return out


def leg_c4(cadmm, torch, args):
    """Headline: the 256 batched scenarios in one handle."""
    prob = workloads.make("c4")
    iters = WORKLOADS["c4"]["iters"]
    h = make_handle(cadmm, prob, args.shape)
    W, n_wg, G = h.launch_config()
    for _ in range(args.warmup):
        h.reset(); h.iterate(iters); h.scales()
    say(f"c4: warmup done, blocks/group={W} workgroups={n_wg} lanes/pair={G}")
    sec = time_solves(h, iters, args.steps, torch)
    code, res = h.solve(0)
    rp, rd = h.history(iters)
    it = np.array([r["iters"] for r in res])
    solves = float((pairs_per_scenario(prob) * it).sum())
    h.reset()
    ph = h.phase_times(iters)
    h.close()
    bl = pair_bytes(prob)
    out = dict(sec=sec, solves=solves, iters=it, res=res, ph=ph, launch=(W, n_wg, G),
               npairs=int(pairs_per_scenario(prob).sum()))
    out["summary"] = residual_summary(prob, res, rp, rd)
    out["roofline"] = roofline(bl, ph[0], measured_traffic("pair_phase_c4", (W, G)), "pair_phase_kernel",
                               overhead_bytes=partial_bytes(n_wg, prob),
                               valu=valu_rate(measured_valu("pair_phase_c4", (W, G)), ph[0]),
                               launch={"blocks_per_group": W, "workgroups": n_wg, "lanes_per_pair": G})
    return out


def leg_plain(cadmm, torch, iters=50, steps=2):
    """The same 256 scenarios as 256 separate handles launched one after
    another on one stream (the plain per-scenario form)."""
    prob = workloads.make("c4")
    S = workloads.n_scenarios(prob)
    plain = [cadmm.Handle(workloads.select_scenarios(prob, [s])) for s in range(S)]
    for h in plain:
        h.reset(); h.iterate(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for h in plain:
            h.reset()
            h.iterate(iters)
            h.scales()
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / steps
    solves = 0.0
    for s, h in enumerate(plain):
        _, res = h.solve(0)
        solves += pairs_per_scenario(workloads.select_scenarios(prob, [s]))[0] * res[0]["iters"]
    for h in plain:
        h.close()
    return dict(sec=tp, solves=solves)


def leg_single(cadmm, torch, name, args, steps=10):
    """One scenario solved to the stopping test (or the iteration cap): the
    time of admm_solve (graph chunks of 16 iterations, done flags read after
    each), the pair solves it ran, the residuals and the per-phase times."""
    prob = workloads.make(name)
    cap = WORKLOADS[name]["iters"]
    h = make_handle(cadmm, prob, args.shape if name == args.workload else "")
    W, n_wg, G = h.launch_config()
    h.reset(); h.solve(cap, check_every=16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.reset()
        code, res = h.solve(cap, check_every=16)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    rp, rd = h.history(cap)
    it = res[0]["iters"]
    npairs = int(pairs_per_scenario(prob).sum())
    h.reset()
    ph = h.phase_times(it)
    h.close()
    bl = pair_bytes(prob)
    return dict(workload=f"{name}: {WORKLOADS[name]['desc']}", pairs_per_iteration=npairs, admm_iterations=it,
                ms_per_solve=sec * 1e3, pair_solves_per_s=npairs * it / sec, admm_iters_per_s=it / sec,
                pair_phase_solves_per_s=npairs / (ph[0] * 1e-3),
                residuals=residual_summary(prob, res, rp, rd),
                phase_ms={"pair": ph[0], "trajectory": ph[1], "multiplier": ph[2], "residual": ph[3]},
                roofline=roofline(bl, ph[0], measured_traffic(f"pair_phase_{name}", (W, G)), "pair_phase_kernel",
                                  overhead_bytes=partial_bytes(n_wg, prob),
                                  launch={"blocks_per_group": W, "workgroups": n_wg, "lanes_per_pair": G}))


def stream_bytes(rp, n_pairs):
    """Algorithmic bytes of one stateless batch: per row read K (dim + 1
    floats), kappa and yhat, write y; per pair read row_ptr and bhat, write
    r, nu and status (2D)."""
    rows = int(rp[-1])
    return 4.0 * rows * (3 + 1 + 1 + 1) + 4.0 * n_pairs * (1 + 3 + 3 + 1 + 1)


def time_batch(cadmm, torch, args, reps, **kw):
    """Mean ms of one pair_qp_batch call (HIP events on torch's current
    stream, the stream the kernels run on) and its last outputs."""
    out = cadmm.pair_qp_batch(*args, 0.1, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = cadmm.pair_qp_batch(*args, 0.1, **kw)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


_STREAM_INPUTS = {}   # the streamed batch, generated once for both forms


def leg_stream(cadmm, torch, n_pairs=1 << 22, reps=5, two_launch=False):
    """The stateless pair-QP entry point streamed over 2^22 pairs of the
    batched 2D shape (about 1.4 GB, beyond the 256 MB Infinity Cache): the
    size at which HBM, not latency, bounds the pair solve. two_launch: the
    form with a workspace, whose second launch resumes the pairs still
    running after three sweeps."""
    key = ("stream", n_pairs)
    if key not in _STREAM_INPUTS:
        rp, K, kap, yh, bh = workloads.pair_batch_c4_shape(n_pairs)
        _STREAM_INPUTS[key] = (rp, [torch.from_numpy(a).to("cuda") for a in (rp, K, kap, yh, bh)])
    rp, args = _STREAM_INPUTS[key]
    kw = {}
    if two_launch:
        kw["work"] = torch.empty(cadmm.pair_qp_batch_workspace_size(n_pairs) + 256, dtype=torch.uint8,
                                 device="cuda")
    ms, (y, r, nu, status) = time_batch(cadmm, torch, args, reps, **kw)
    bytes_launch = stream_bytes(rp, n_pairs)
    st = status.cpu().numpy()
    name = "pair_qp_batch_stream2" if two_launch else "pair_qp_batch_stream"
    out = dict(workload=f"{n_pairs} stateless pair QPs of the batched 2D shape ({int(rp[-1])} rows, 5-16 per pair)"
                        + (", two-launch form" if two_launch else ", one launch"),
               ms_per_launch=ms, pair_solves_per_s=n_pairs / (ms * 1e-3),
               sweeps_mean=float(st[st >= 0].mean()), budget_hits=int((st < 0).sum()))
    if two_launch:
        out["queued_after_3_sweeps"] = int((st > 3).sum())
        out["gb_per_s"] = bytes_launch / (ms * 1e-3) / 1e9
    else:
        out["roofline"] = roofline(bytes_launch, ms, measured_traffic(name, kernel="pair_qp_batch_kernel"),
                                   "pair_qp_batch_kernel",
                                   valu=valu_rate(measured_valu(name, kernel="pair_qp_batch_kernel"), ms))
    return out


def leg_lemke(cadmm, torch, n_pairs=1 << 18, reps=3):
    """A/B of the two pair solvers on the same stateless batch (2^18 pairs of
    the batched 2D shape): the dual Newton method against the Sec. IV-C route
    (elimination, LCP, Lemke pivoting), and the largest difference of their
    duals scaled by the pair's row norms."""
    rp, K, kap, yh, bh = workloads.pair_batch_c4_shape(n_pairs, seed=5)
    args = [torch.from_numpy(a).to("cuda") for a in (rp, K, kap, yh, bh)]
    ms_n, (yn, _, _, st_n) = time_batch(cadmm, torch, args, reps)
    ms_l, (yl, _, _, st_l) = time_batch(cadmm, torch, args, reps, solver=cadmm.CADMM_PAIR_LEMKE)
    stl = st_l.cpu().numpy()
    return dict(workload=f"{n_pairs} stateless pair QPs of the batched 2D shape", ms_newton=ms_n, ms_lemke=ms_l,
                lemke_over_newton=ms_l / ms_n, lemke_pivots_mean=float(stl[stl >= 0].mean()),
                lemke_failures=int((stl < 0).sum()), newton_failures=int((st_n < 0).sum().item()),
                max_abs_dual_difference=float((yn - yl).abs().max().item()))


def leg_loop(cadmm, torch):
    """The receding-horizon closed loop of the synthetic Sec. V-A scene (250
    control cycles of 0.1 s, T = 16, 32 obstacles, a 20 x 20 x 6 m sensing
    window): wall time per control loop (new set-up when the sensed set
    changes, x0 and reference update, shifted warm start, admm_solve with at
    least 5 iterations, state read back), one warm-up run first."""
    from paper_2406_07048_amd.closed_loop import ClosedLoop
    scene = workloads.closed_loop_scene()
    cycles = len(scene["ref"]) - 1
    ClosedLoop(scene).run(20)
    loop = ClosedLoop(scene)
    out = loop.run(cycles)
    loop.close()
    recs = out["records"]
    t = np.array([r["setup_s"] + r["solve_s"] for r in recs]) * 1e3
    ts = np.array([r["solve_s"] for r in recs if not r["setup"]]) * 1e3
    it = np.array([r["iters"] for r in recs])
    pairs = np.array([r["pairs"] for r in recs])
    return dict(workload="closed loop: 250 cycles of 0.1 s, quadrotor box, 32 pillars in 70x20x6 m, 20x20x6 m "
                         "sensing, T=16, sigma=300",
                ms_per_control_loop=float(t.mean()), ms_per_control_loop_max=float(t.max()),
                ms_per_solve_without_setup=float(ts.mean()) if ts.size else None,
                setups=int(sum(r["setup"] for r in recs)), iterations_mean=float(it.mean()),
                iterations_max=int(it.max()), pairs_mean=float(pairs.mean()), pairs_max=int(pairs.max()),
                goal_distance_m=float(np.linalg.norm(out["x"][-1, :3] - scene["ref"][-1, :3])),
                min_alpha=float(min(r["min_alpha"] for r in recs)))


def leg_grad(cadmm, torch, steps=3, iters=100, every=10):
    """Reverse pass of the 3D configuration unrolled over 100 iterations with
    a checkpoint every 10: wall time of admm_backward (segment replay +
    adjoint kernels) against the forward run that records the checkpoints,
    and against a plain 100-iteration forward solve."""
    prob = workloads.make("c3")
    h = cadmm.Handle(prob)
    nbytes = h.grad_workspace_size(iters, every)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def plain():
        h.reset()
        h.iterate(iters)

    def rec():
        h.reset()
        h.record(iters, every)

    plain(); rec(); h.backward()
    t_plain = timed(plain)
    t_rec = timed(rec)
    t_bwd = timed(lambda: h.backward())
    h.close()
    n_faces = len(prob["obs_d"])
    return dict(workload=f"3D quadrotor (3 boxes), 200 hull polyhedra, N=40, {iters} unrolled iterations, "
                         f"checkpoint every {every}; gradient w.r.t. {n_faces} obstacle offsets and the "
                         f"{prob['n_s']}-dim initial state",
                forward_ms=t_rec * 1e3, plain_solve_ms=t_plain * 1e3, backward_ms=t_bwd * 1e3,
                backward_forward_ratio=t_bwd / t_rec, grad_workspace_mb=nbytes / 1e6)


def leg_cpu(prob, iters, budget_s=25.0, min_s=10.0):
    """The FP64 oracle (OpenMP over the pair QPs) on the host cores, on the
    headline workload: its scenarios in order, each initialised and iterated
    like the GPU run, in chunks of 16 scenarios, until at least min_s seconds
    (starting over after the last scenario) or the budget is spent."""
    import oracle
    cores = oracle.set_threads(0)
    S = workloads.n_scenarios(prob)
    pps = pairs_per_scenario(prob)
    solves = 0.0
    done = 0
    t0 = time.perf_counter()
    chunk = 16
    s0 = 0
    while True:
        idx = list(range(s0, min(S, s0 + chunk)))
        P = oracle.Problem(workloads.select_scenarios(prob, idx))
        st = P.init_state()
        hist = P.run(st, iters)
        solves += float((pps[idx] * hist["iters"]).sum())
        done += len(idx)
        s0 = 0 if s0 + chunk >= S else s0 + chunk
        el = time.perf_counter() - t0
        if el >= budget_s or (el >= min_s and s0 == 0):
            break
    el = time.perf_counter() - t0
    return dict(value=solves / el, unit="pair-QP solves/s", cores=int(cores), kind="oracle",
                sample=f"{done} scenario solves of the same batched workload ({S} scenarios, init + {iters} "
                       f"iterations each, {int(solves)} pair QPs), {el:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=("c4",),
                    help="the headline workload (the 256 batched scenarios)")
    ap.add_argument("--legs", default=",".join(ALL_LEGS),
                    help="comma list of legs to run: " + ",".join(ALL_LEGS))
    ap.add_argument("--shape", default="", metavar="W,G",
                    help="fix the pair-kernel launch shape of the headline handle (blocks per workgroup W, lanes "
                         "per pair G) instead of autotuning it; the counter runs behind profiles/ use the "
                         "shape the autotuner picks, so that their dispatches are the bench's")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hashes of the profiled kernels' sources and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one plain device-to-device copy of MIB MiB (the reference for the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.source_hash:
        print(json.dumps({k: kernel_source_hash(k) for k in KERNEL_SOURCES}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build runs on a single GPU; the batched scenarios would "
              f"shard across GPUs with no exchange); got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    legs = [l for l in args.legs.split(",") if l]
    for l in legs:
        if l not in ALL_LEGS:
            ap.error(f"unknown leg {l}")
    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return
    import paper_2406_07048_amd as cadmm

    prob = workloads.make("c4")
    iters = WORKLOADS["c4"]["iters"]
    out = {"metric": METRIC, "value": None, "unit": "pair-QP solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"c4: {WORKLOADS['c4']['desc']}", "scenarios": workloads.n_scenarios(prob),
                      "admm_iterations": iters, "parallelism": "single GPU"}}
    if "c4" in legs:
        c4 = leg_c4(cadmm, torch, args)
        sec = c4["sec"]
        out["value"] = c4["solves"] / sec
        out["ms_per_step"] = sec * 1e3
        out["config"]["pairs_per_iteration"] = c4["npairs"]
        out["pair_solves_per_step"] = c4["solves"]
        out["admm_iters_per_s"] = iters / sec
        out["scenario_iters_per_s"] = float(c4["iters"].sum()) / sec
        out["pair_phase_solves_per_s"] = c4["npairs"] / (c4["ph"][0] * 1e-3)
        out["residuals"] = c4["summary"]
        out["phase_ms"] = dict(zip(("pair", "trajectory", "multiplier", "residual"), c4["ph"]))
        out["roofline"] = c4["roofline"]
        if "plain" in legs:
            say("plain: 256 separate handles")
            pl = leg_plain(cadmm, torch, iters)
            out["batched_vs_plain"] = {"plain_pair_solves_per_s": pl["solves"] / pl["sec"],
                                       "plain_ms_per_step": pl["sec"] * 1e3,
                                       "speedup": pl["sec"] / sec * (c4["solves"] / max(pl["solves"], 1.0))}
    for name in ("c2", "c3", "c2tv", "c2sqp", "c3sqp", "c2b"):
        if name in legs:
            say(f"{name}: single scenario to the stopping test")
            out[name] = leg_single(cadmm, torch, name, args)
    if "stream" in legs:
        say("stream: stateless pair QPs (2^22)")
        out["stream"] = leg_stream(cadmm, torch)
    if "stream2" in legs:
        say("stream2: stateless pair QPs (2^22), two-launch form")
        out["stream2"] = leg_stream(cadmm, torch, two_launch=True)
    if "lemke" in legs:
        say("lemke: Newton vs Lemke pair solvers (2^18)")
        out["lemke"] = leg_lemke(cadmm, torch)
    if "loop" in legs:
        say("loop: receding-horizon closed loop (250 cycles)")
        out["closed_loop"] = leg_loop(cadmm, torch)
    if "grad" in legs:
        say("grad: reverse pass (3D, 100 unrolled iterations)")
        out["differentiation"] = leg_grad(cadmm, torch)
    if "cpu" in legs:
        say("cpu: FP64 oracle on the headline workload")
        out["cpu_baseline"] = leg_cpu(prob, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
