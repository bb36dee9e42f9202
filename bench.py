#!/usr/bin/env python3
"""Benchmark of the ADMM collision-avoidance hot path on one MI355X.

A step is one complete solve of the workload with inputs resident in HBM:
reset to the initial iterate (obstacle-free LQ trajectory, scale-LP
certificates), the ADMM iterations (pair QPs, trajectory QP, multiplier
update, residual test, all inside a HIP graph) and the final scale
certificate at the last trajectory. The headline value is pair-QP solves per
second over the timed steps; ADMM iterations per second and the residuals
reached are reported beside it, together with the batched-vs-plain comparison
on 256 scenarios, the pair kernel's roofline figure and the FP64 oracle timed
on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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
KERNEL_SOURCES = ("paper_2406_07048_amd/csrc/cadmm_kernels.hip", "paper_2406_07048_amd/csrc/cadmm_device.h",
                  "paper_2406_07048_amd/csrc/cadmm_internal.h")

WORKLOADS = {
    "c2": dict(desc="2D cab+trailer (2 parts x 4 faces), 40 hull obstacles (3-10 faces), N=50, "
                    "4000 pair QPs/iteration, 200 ADMM iterations, sigma=300", iters=200),
    "c3": dict(desc="3D quadrotor (3 boxes), 200 hull polyhedra (6-20 faces), N=40, "
                    "24000 pair QPs/iteration, 200 ADMM iterations, sigma=300", iters=200),
    "c1": dict(desc="2D rectangle, 3 obstacles, N=20, 60 pair QPs/iteration, 50 ADMM iterations", iters=50),
    "c4": dict(desc="256 2D scenarios, obstacles U{10..80}, faces U{3..12}, N=50, 50 ADMM iterations", iters=50),
}


def pair_bytes(prob, n_wg, nc):
    """Algorithmic HBM bytes of one pair-phase launch: each pair reads its
    previous duals (n floats), writes the new ones (n floats) and reads its
    multipliers (1 + dim floats); each workgroup writes nc x 64 floats of
    per-step contribution sums. Geometry and poses are cache-resident."""
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
    N, dim = prob["N"], prob["dim"]
    return 4.0 * (2 * tot + len(sc) * N * (1 + dim)) + 4.0 * n_wg * nc * 64


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(name, launch=None):
    """HBM bytes per launch of a kernel from the committed counter summary
    profiles/<name>_hbm_traffic.txt (FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by what the same counters read for a plain copy of known size).
    None when the summary is missing, was taken from other kernel sources or,
    given launch = (blocks per workgroup, lanes per pair), at another launch
    shape."""
    path = os.path.join(ROOT, "profiles", f"{name}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    if launch is not None and kv.get("launch") != f"{launch[0]},{launch[1]}":
        return None
    return float(kv["traffic_bytes_per_launch"])


def time_solves(h, iters, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.reset()
        h.iterate(iters)
        h.scales()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_baseline(prob, iters, budget_s=12.0):
    """The FP64 oracle on the host cores over a bounded sample of the same
    solve: whole solves (init + iterations) repeated until the budget."""
    import oracle
    cores = oracle.set_threads(0)
    P = oracle.Problem(prob)
    n = 0
    pairs = 0
    t0 = time.perf_counter()
    while True:
        st = P.init_state()
        hist = P.run(st, iters)
        n += 1
        pairs += P.n_blocks * prob["N"] * int(hist["iters"].max())
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return dict(value=pairs / el, unit="pair-QP solves/s", cores=int(cores), kind="oracle",
                sample=f"{n} complete FP64 oracle solve(s) of the same workload "
                       f"(init + {iters} iterations), {el:.1f} s wall")


def batched_vs_plain(cadmm, torch, steps=2, iters=50):
    """256 scenarios of the 2D batched configuration in one handle vs 256
    separate handles launched one after another on one stream."""
    prob = workloads.make("c4")
    S = len(prob["obs_ptr"]) - 1
    hb = cadmm.Handle(prob)
    time_solves(hb, iters, 1, torch)
    tb = time_solves(hb, iters, steps, torch)
    _, nb, npairs, _ = cadmm.cadmm_workspace_size(prob)
    wb = hb.launch_config()
    # HBM roofline of the batched pair phase (the size where HBM, not launch
    # latency, bounds it), from HIP events on the handle's stream
    hb.reset()
    ph = hb.phase_times(iters)
    nq = prob["dim"] + (1 if prob["dim"] == 2 else 3)
    bytes_launch = pair_bytes(prob, wb[1], nq * (nq + 1) // 2 + nq)
    gbs = bytes_launch / (ph[0] * 1e-3) / 1e9
    hb.close()
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
    for h in plain:
        h.close()
    solves = npairs * iters
    return dict(workload=f"{S} 2D scenarios, obstacles U{{10..80}}, faces U{{3..12}}, N=50, {npairs} pair QPs "
                         f"per iteration, {iters} iterations",
                batched_pair_solves_per_s=solves / tb, plain_pair_solves_per_s=solves / tp,
                batched_ms_per_solve=tb * 1e3, plain_ms_per_solve=tp * 1e3, speedup=tp / tb,
                batched_blocks_per_group=wb[0], batched_lanes_per_pair=wb[2],
                pair_phase_ms=ph[0], pair_phase_solves_per_s=npairs / (ph[0] * 1e-3),
                roofline={"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic("pair_phase_c4", (wb[0], wb[2])),
                          "kernel": "pair_phase_kernel", "bytes_per_launch": bytes_launch})


def stream_batch(cadmm, torch, n_pairs=1 << 22, reps=5):
    """The stateless pair-QP entry point streamed over 2^22 pairs of the
    batched 2D shape (about 1.4 GB, beyond the 256 MB Infinity Cache): the
    size at which HBM, not latency, bounds the pair solve. HIP events on the
    stream the kernel runs on (torch's current stream)."""
    rp, K, kap, yh, bh = workloads.pair_batch_c4_shape(n_pairs)
    args = [torch.from_numpy(a).to("cuda") for a in (rp, K, kap, yh, bh)]
    y, r, status = cadmm.pair_qp_batch(*args, 0.1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        cadmm.pair_qp_batch(*args, 0.1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rows = int(rp[-1])
    # read K, kappa, yhat, write y (per row); read bhat, row_ptr, write r, status (per pair)
    bytes_launch = 4.0 * rows * (3 + 1 + 1 + 1) + 4.0 * n_pairs * (3 + 1 + 3 + 1)
    gbs = bytes_launch / (ms * 1e-3) / 1e9
    st = status.cpu().numpy()
    return dict(workload=f"{n_pairs} stateless pair QPs of the batched 2D shape ({rows} rows, 5-16 per pair)",
                ms_per_launch=ms, pair_solves_per_s=n_pairs / (ms * 1e-3),
                sweeps_mean=float(st[st >= 0].mean()), budget_hits=int((st < 0).sum()),
                roofline={"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "pair_qp_batch_kernel",
                          "bytes_per_launch": bytes_launch})


def differentiation(cadmm, torch, steps=3, iters=100, every=10):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--shape", default="", metavar="W,G",
                    help="fix the pair-kernel launch shape of the main workload (blocks per workgroup W, lanes "
                         "per pair G) instead of autotuning it; the counter runs behind profiles/ use the "
                         "shape the autotuner picks, so that their dispatches are the bench's")
    ap.add_argument("--source-hash", action="store_true", help="print the hash of the kernel sources and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one plain device-to-device copy of MIB MiB (the reference for the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
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

    wl = WORKLOADS[args.workload]
    prob = workloads.make(args.workload)
    iters = wl["iters"]
    if args.shape:
        sw, sg = (int(v) for v in args.shape.split(","))
        h = cadmm.Handle(prob, waves_per_group=sw, lanes_per_pair=sg)
    else:
        h = cadmm.Handle(prob)
    W, n_wg, G = h.launch_config()
    _, nb, npairs, yf = cadmm.cadmm_workspace_size(prob)
    for _ in range(args.warmup):
        h.reset(); h.iterate(iters); h.scales()
    print(f"[bench] {args.workload}: warmup done, blocks/group={W} workgroups={n_wg} lanes/pair={G}",
          file=sys.stderr, flush=True)
    sec = time_solves(h, iters, args.steps, torch)
    code, res = h.solve(0)
    rp, rd = h.history(iters)
    it_done = max(r["iters"] for r in res)
    reached = None
    for k in range(rp.shape[0]):
        if rp[k, 0] <= prob["eps_pri"] and rd[k, 0] <= prob["eps_dual"]:
            reached = k + 1
            break
    solves = npairs * it_done
    # roofline figure of the dominant kernel (pair phase): HIP events recorded
    # around each launch's own execution on the handle's stream, over the
    # same iterations as the timed solves (the first iterations carry more
    # Newton sweeps than the later ones, so a shorter window would differ)
    h.reset()
    ph = h.phase_times(it_done)
    nq = prob["dim"] + (1 if prob["dim"] == 2 else 3)
    nc = nq * (nq + 1) // 2 + nq
    bytes_launch = pair_bytes(prob, n_wg, nc)
    achieved = bytes_launch / (ph[0] * 1e-3) / 1e9
    out = {
        "metric": "pair-QP solves/sec & ADMM iters/sec at res 1e-4 (batched vs plain); backward/forward ratio",
        "value": solves / sec,
        "unit": "pair-QP solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "pairs_per_iteration": npairs,
                   "admm_iterations": it_done, "parallelism": "single GPU"},
        "admm_iters_per_s": it_done / sec,
        "pair_phase_solves_per_s": npairs / (ph[0] * 1e-3),
        "residuals": {"r_pri": res[0]["r_pri"], "r_dual": res[0]["r_dual"], "first_iter_at_1e-4": reached,
                      "converged": res[0]["converged"], "min_alpha": res[0]["min_alpha"], "cost": res[0]["cost"]},
        "phase_ms": {"pair": ph[0], "trajectory": ph[1], "multiplier": ph[2], "residual": ph[3]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"pair_phase_{args.workload}") if args.workload == "c2" else None,
                     "kernel": "pair_phase_kernel", "bytes_per_launch": bytes_launch,
                     "launch": {"blocks_per_group": W, "workgroups": n_wg, "lanes_per_pair": G}},
    }
    h.close()
    if not args.no_batched:
        print("[bench] batched vs plain (256 scenarios)", file=sys.stderr, flush=True)
        out["batched"] = batched_vs_plain(cadmm, torch)
    if not args.no_stream:
        print("[bench] streaming stateless pair QPs (2^22)", file=sys.stderr, flush=True)
        out["stream"] = stream_batch(cadmm, torch)
    if not args.no_grad:
        print("[bench] reverse pass (3D, 100 unrolled iterations)", file=sys.stderr, flush=True)
        out["differentiation"] = differentiation(cadmm, torch)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (FP64 oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
