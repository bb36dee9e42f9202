"""Receding-horizon closed loop on the library (the use of Sec. V-A: one MPC
solve per control cycle of dt, the first input applied to the plant).

Per cycle k:
  1. the obstacles the robot senses at its measured state (a window around
     it); when that set changes the handle is set up anew for it;
  2. the measured state as x0 (admm_set_params) and the reference samples
     k .. k + N (admm_set_reference);
  3. a warm start from the previous cycle's solution shifted by one step
     (admm_set_state): states and inputs, and the duals and multipliers of
     every pair block whose obstacle is still sensed; pair blocks of newly
     sensed obstacles start from the scale-LP certificates at the warm
     trajectory with zero multipliers (admm_reset_duals);
  4. the ADMM solve (admm_solve to the stopping test of Sec. IV-B, or a fixed
     number of iterations);
  5. the first input applied to the plant: the nonlinear model stepped on
     the host in FP64 (cadmm_model_step).

Only the ABI is called; the solve runs in the library's kernels."""
from __future__ import annotations

import time

import numpy as np

import workloads

from . import Handle, model_step


class ClosedLoop:
    """The closed loop of one scene (workloads.closed_loop_scene).

    max_iters, check_every: admm_solve's iteration cap and flag interval;
    min_iters: iterations run before the stopping test is looked at (a warm
    start can pass the test of Sec. IV-B at once, which only sees the pair
    variables, while the SQP step of the trajectory still moves);
    fixed_iters: run exactly this many iterations per cycle instead (no
    stopping test); shape: (pair blocks per workgroup, lanes per pair QP),
    fixed so that a set-up does not autotune."""

    def __init__(self, scene, max_iters=100, check_every=8, min_iters=5, fixed_iters=None, shape=(1, 4)):
        self.scene = scene
        self.max_iters = int(max_iters)
        self.min_iters = int(min_iters)
        self.count = 0            # iterations the current handle has run
        self.check_every = int(check_every)
        self.fixed_iters = fixed_iters
        self.shape = shape
        self.N = scene["base"]["N"]
        self.base = scene["base"]
        self.h = None
        self.ids = None
        self.prob = None
        self.prev = None          # previous cycle's solution (host arrays) and its block keys

    def _blocks(self, prob, ids):
        """(part, global obstacle) -> (y offset, rows, block index) of the
        canonical layout of a cycle problem."""
        sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
        return {(int(part[b]), int(ids[obs[b]])): (int(yoff[b]), int(nrow[b]), b) for b in range(len(sc))}

    def _warm_state(self, x_meas, new_blocks, state0, carry=True):
        """Warm start from the previous solution, shifted one step; with
        carry the pair iterate of every block whose obstacle was sensed
        before, else state0's."""
        N, dim = self.N, self.base["dim"]
        x = np.empty((1, N + 1, self.base["n_s"]))
        u = np.empty((1, N, self.base["n_u"]))
        px, pu = self.prev["x"], self.prev["u"]
        x[0, 0] = x_meas
        x[0, 1:N] = px[0, 2:N + 1]
        x[0, N] = px[0, N]
        u[0, :N - 1] = pu[0, 1:]
        u[0, N - 1] = pu[0, N - 1]
        if not carry:
            return dict(x=x, u=u)
        y, zeta, xi = state0["y"].copy(), state0["zeta"].copy(), state0["xi"].copy()
        old = self.prev["blocks"]
        for key, (off, n, b) in new_blocks.items():
            if key not in old:
                continue
            ooff, on, ob = old[key]
            yo = self.prev["y"][ooff:ooff + on * N].reshape(on, N)
            yn = np.concatenate([yo[:, 1:], yo[:, -1:]], axis=1)
            y[off:off + n * N] = yn.ravel()
            zo = self.prev["zeta"][ob * N:(ob + 1) * N]
            zeta[b * N:(b + 1) * N] = np.concatenate([zo[1:], zo[-1:]])
            xo = self.prev["xi"][ob * dim * N:(ob + 1) * dim * N].reshape(dim, N)
            xi[b * dim * N:(b + 1) * dim * N] = np.concatenate([xo[:, 1:], xo[:, -1:]], axis=1).ravel()
        return dict(x=x, u=u, y=y, zeta=zeta, xi=xi)

    def step(self, x_meas, k):
        """One control cycle at the measured state x_meas; returns the input
        applied and the cycle's record."""
        import torch
        rec = {}
        t0 = time.perf_counter()
        ids = workloads.sensed(self.scene, x_meas[:3])
        if ids != self.ids:
            if self.h is not None:
                self.h.close()
            self.prob = workloads.cycle_problem(self.scene, ids, x_meas, k)
            if self.fixed_iters is not None:
                self.prob.update(eps_pri=-1.0, eps_dual=-1.0)     # no stopping test
            self.h = Handle(self.prob, waves_per_group=self.shape[0], lanes_per_pair=self.shape[1])
            self.ids = ids
            self.count = 0
            rec["setup"] = True
        else:
            self.h.set_params(x0=x_meas[None])
            self.h.set_reference(workloads.reference_window(self.scene, k))
            rec["setup"] = False
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        blocks = self._blocks(self.prob, ids)
        if self.prev is not None:
            ws = self._warm_state(x_meas, blocks, {a: self.prev[a] for a in ("y", "zeta", "xi")}, carry=False)
            if rec["setup"]:
                # newly sensed obstacles: the scale-LP certificates at the warm
                # trajectory (admm_reset_duals); the others carried
                self.h.set_state(x=ws["x"], u=ws["u"])
                self.h.reset_duals()
                st0 = self.h.get_state_host()
            else:
                st0 = {a: self.prev[a] for a in ("y", "zeta", "xi")}
            self.h.set_state(**self._warm_state(x_meas, blocks, st0))
        if self.fixed_iters is not None:
            self.h.iterate(int(self.fixed_iters))
            iters = int(self.fixed_iters)
            min_alpha = None
        else:
            # the handle counts iterations since its set-up, stopped ones excluded
            if self.min_iters:
                self.h.iterate(self.min_iters)
            code, res = self.h.solve(self.max_iters - self.min_iters, check_every=self.check_every)
            iters = res[0]["iters"] - self.count
            self.count = res[0]["iters"]
            min_alpha = res[0]["min_alpha"]
        st = self.h.get_state_host()
        t2 = time.perf_counter()
        u0 = st["u"][0, 0].copy()
        self.prev = dict(x=st["x"], u=st["u"], y=st["y"], zeta=st["zeta"], xi=st["xi"], blocks=blocks)
        rec.update(k=k, sensed=len(ids), pairs=len(blocks) * self.N, iters=iters, min_alpha=min_alpha,
                   setup_s=t1 - t0, solve_s=t2 - t1, u0=u0, x_pred=st["x"][0].copy())
        return u0, rec

    def run(self, cycles, k0=0, x_start=None):
        """Run cycles k0 .. k0 + cycles - 1 from x_start (default: the scene's
        start); returns the applied inputs, the plant states and the records."""
        x = np.array(self.scene["x_start"] if x_start is None else x_start, dtype=np.float64)
        xs, us, recs = [x.copy()], [], []
        par = self.base["model_par"]
        for k in range(k0, k0 + cycles):
            u0, rec = self.step(x, k)
            x = model_step(self.base["model"], par, x, u0)
            xs.append(x.copy())
            us.append(u0)
            recs.append(rec)
        return dict(x=np.array(xs), u=np.array(us), records=recs)

    def close(self):
        if self.h is not None:
            self.h.close()
            self.h = None
