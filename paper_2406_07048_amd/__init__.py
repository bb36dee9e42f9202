"""MI355X (gfx950) ADMM collision avoidance for polyhedral robots and obstacles.

Thin Python binding of the C ABI in ``include/cadmm.h`` (method of
"GPU-Accelerated Optimization-Based Collision Avoidance", arXiv 2406.07048).
Every step of the path runs in the HIP kernels of ``_libcadmm.so``; this module
only marshals arguments. PyTorch provides device memory (the caller-owned
workspace and I/O tensors) and the current HIP stream. There is no CPU
fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_libcadmm.so")
_lib = None

CADMM_OK, CADMM_INVALID, CADMM_DEVICE, CADMM_WORKSPACE, CADMM_NOT_CONVERGED = 0, 1, 2, 3, 4

_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class CadmmDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n_s", ctypes.c_int), ("n_u", ctypes.c_int), ("N", ctypes.c_int),
        ("n_parts", ctypes.c_int),
        ("part_face_ptr", _ip), ("part_A", _dp), ("part_b", _dp), ("part_off", _dp),
        ("n_scen", ctypes.c_int),
        ("obs_ptr", _ip), ("obs_face_ptr", _ip), ("obs_C", _dp), ("obs_d", _dp),
        ("A_dyn", _dp), ("B_dyn", _dp), ("c_dyn", _dp),
        ("pos_idx", _ip), ("att_idx", _ip), ("att_kind", ctypes.c_int),
        ("Q_s", _dp), ("Q_u", _dp), ("x_ref", _dp), ("x0", _dp),
        ("sigma", ctypes.c_double), ("eps_prox", ctypes.c_double),
        ("eps_pri", ctypes.c_double), ("eps_dual", ctypes.c_double),
        ("max_sweeps", ctypes.c_int), ("waves_per_group", ctypes.c_int), ("lanes_per_pair", ctypes.c_int),
        ("dyn_t_stride", ctypes.c_int), ("dyn_s_stride", ctypes.c_int), ("model", ctypes.c_int),
        ("model_par", ctypes.c_double * 8),
        ("s_min", _dp), ("s_max", _dp), ("u_min", _dp), ("u_max", _dp),
    ]


CADMM_MODEL_LINEAR, CADMM_MODEL_BICYCLE, CADMM_MODEL_QUADROTOR = 0, 1, 2


class CadmmResult(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int), ("converged", ctypes.c_int),
        ("r_pri", ctypes.c_float), ("r_dual", ctypes.c_float),
        ("cost", ctypes.c_float), ("min_alpha", ctypes.c_float),
        ("unconverged_pairs", ctypes.c_int),
        ("active_bounds", ctypes.c_int),
    ]


class CadmmPairBatch(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int), ("dim", ctypes.c_int),
        ("row_ptr", _vp), ("K", _vp), ("kappa", _vp), ("yhat", _vp), ("bhat", _vp),
        ("eps", ctypes.c_float), ("max_sweeps", ctypes.c_int),
        ("y", _vp), ("r", _vp), ("nu", _vp), ("status", _vp), ("solver", ctypes.c_int),
        ("work", _vp), ("work_bytes", ctypes.c_size_t),
    ]


CADMM_PAIR_NEWTON, CADMM_PAIR_LEMKE = 0, 1


class CadmmScaleBatch(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int), ("dim", ctypes.c_int),
        ("a_ptr", _vp), ("A", _vp), ("b", _vp), ("o_ptr", _vp), ("Cp", _vp), ("dp", _vp),
        ("alpha", _vp), ("lam", _vp), ("mu", _vp), ("status", _vp),
    ]


# every symbol the header declares, with its ctypes signature
_SIGNATURES = {
    "cadmm_workspace_size": (ctypes.c_int, [ctypes.POINTER(CadmmDesc), ctypes.POINTER(ctypes.c_size_t), _ip,
                                            ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
    "collision_admm_setup": (ctypes.c_int, [ctypes.POINTER(CadmmDesc), _vp, ctypes.c_size_t, _vp,
                                            ctypes.POINTER(_vp)]),
    "admm_iterate": (ctypes.c_int, [_vp, ctypes.c_int]),
    "admm_solve": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(CadmmResult)]),
    "admm_reset": (ctypes.c_int, [_vp]),
    "admm_get_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "admm_set_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "admm_get_history": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "admm_scales": (ctypes.c_int, [_vp, _vp]),
    "admm_phase_times": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "admm_launch_config": (ctypes.c_int, [_vp, _ip, _ip, _ip]),
    "admm_set_params": (ctypes.c_int, [_vp, _dp, _dp]),
    "admm_set_reference": (ctypes.c_int, [_vp, _dp]),
    "admm_reset_duals": (ctypes.c_int, [_vp]),
    "cadmm_model_step": (ctypes.c_int, [ctypes.c_int, _dp, _dp, _dp, _dp]),
    "admm_grad_workspace_size": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "admm_record": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp]),
    "admm_backward": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_float, _vp, _vp]),
    "collision_admm_destroy": (None, [_vp]),
    "pair_qp_batch": (ctypes.c_int, [ctypes.POINTER(CadmmPairBatch), _vp]),
    "pair_qp_batch_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "pair_qp_batch_noalloc": (ctypes.c_int, [ctypes.POINTER(CadmmPairBatch), _vp]),
    "pair_scale_batch": (ctypes.c_int, [ctypes.POINTER(CadmmScaleBatch), _vp]),
    "cadmm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cadmm_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (build it with __graft_entry__.build())")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so both share one runtime, device list and streams
        _torch()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CadmmError(RuntimeError):
    def __init__(self, code, where):
        L = lib()
        super().__init__(f"{where}: {L.cadmm_strerror(code).decode()} ({L.cadmm_last_error().decode()})")
        self.code = code


def _check(code, where, allow=(CADMM_OK,)):
    if code not in allow:
        raise CadmmError(code, where)
    return code


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(st.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class _DescHolder:
    """Contiguous host copies backing a CadmmDesc for the duration of a call."""

    def __init__(self, prob, max_sweeps=0, waves_per_group=0, lanes_per_pair=0):
        keep = {}

        def dbl(name):
            a = np.ascontiguousarray(prob[name], dtype=np.float64)
            keep[name] = a
            return a.ctypes.data_as(_dp)

        def i32(name):
            a = np.ascontiguousarray(prob[name], dtype=np.int32)
            keep[name] = a
            return a.ctypes.data_as(_ip)

        d = CadmmDesc()
        d.dim, d.n_s, d.n_u, d.N = int(prob["dim"]), int(prob["n_s"]), int(prob["n_u"]), int(prob["N"])
        d.n_parts = len(prob["part_face_ptr"]) - 1
        d.part_face_ptr = i32("part_face_ptr")
        d.part_A, d.part_b, d.part_off = dbl("part_A"), dbl("part_b"), dbl("part_off")
        d.n_scen = len(prob["obs_ptr"]) - 1
        d.obs_ptr, d.obs_face_ptr = i32("obs_ptr"), i32("obs_face_ptr")
        d.obs_C, d.obs_d = dbl("obs_C"), dbl("obs_d")
        d.A_dyn, d.B_dyn, d.c_dyn = dbl("A_dyn"), dbl("B_dyn"), dbl("c_dyn")
        d.pos_idx, d.att_idx = i32("pos_idx"), i32("att_idx")
        d.att_kind = int(prob["att_kind"])
        d.Q_s, d.Q_u, d.x_ref, d.x0 = dbl("Q_s"), dbl("Q_u"), dbl("x_ref"), dbl("x0")
        d.sigma, d.eps_prox = float(prob["sigma"]), float(prob["eps_prox"])
        d.eps_pri, d.eps_dual = float(prob["eps_pri"]), float(prob["eps_dual"])
        d.max_sweeps, d.waves_per_group = int(max_sweeps), int(waves_per_group)
        d.lanes_per_pair = int(lanes_per_pair)
        d.dyn_t_stride = int(prob.get("dyn_ts", 0))
        d.dyn_s_stride = int(prob.get("dyn_ss", 0))
        # the library reads n_models models from these host arrays
        n_models = (d.n_scen - 1) * max(d.dyn_s_stride, 0) + (d.N - 1) * max(d.dyn_t_stride, 0) + 1
        for name, per in (("A_dyn", d.n_s * d.n_s), ("B_dyn", d.n_s * d.n_u), ("c_dyn", d.n_s)):
            if keep[name].size < n_models * per:
                raise ValueError(f"{name} holds {keep[name].size // per} models, the strides need {n_models}")
        d.model = int(prob.get("model", CADMM_MODEL_LINEAR))
        for i, v in enumerate(prob.get("model_par", ())):
            d.model_par[i] = float(v)
        for name, n in (("s_min", d.n_s), ("s_max", d.n_s), ("u_min", d.n_u), ("u_max", d.n_u)):
            if prob.get(name) is not None:
                if np.asarray(prob[name]).size != n:
                    raise ValueError(f"{name} must hold {n} values")
                setattr(d, name, dbl(name))
        self.desc = d
        self.keep = keep


def cadmm_workspace_size(prob):
    """(bytes, n_blocks, n_pairs, y_floats) of a problem; validates it."""
    h = _DescHolder(prob)
    nbytes = ctypes.c_size_t()
    nb = ctypes.c_int()
    npairs = ctypes.c_longlong()
    nyf = ctypes.c_longlong()
    _check(lib().cadmm_workspace_size(ctypes.byref(h.desc), ctypes.byref(nbytes), ctypes.byref(nb),
                                      ctypes.byref(npairs), ctypes.byref(nyf)), "cadmm_workspace_size")
    return nbytes.value, nb.value, npairs.value, nyf.value


class Handle:
    """A problem set up on the device (collision_admm_setup) with its workspace."""

    def __init__(self, prob, device="cuda", stream=None, max_sweeps=0, waves_per_group=0, lanes_per_pair=0):
        torch = _torch()
        self.prob = prob
        holder = _DescHolder(prob, max_sweeps, waves_per_group, lanes_per_pair)
        nbytes, self.n_blocks, self.n_pairs, self.y_floats = cadmm_workspace_size(prob)
        self.n_scen = len(prob["obs_ptr"]) - 1
        self.dim, self.N = int(prob["dim"]), int(prob["N"])
        self.n_s, self.n_u = int(prob["n_s"]), int(prob["n_u"])
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib().collision_admm_setup(ctypes.byref(holder.desc), ctypes.c_void_p(self._ws_ptr),
                                          nbytes, _stream_ptr(self.stream), ctypes.byref(h)),
               "collision_admm_setup")
        self._h = h
        # the initial duals of setup (scale-LP certificates at the
        # descriptor's own offsets and initial states): the default y^0 of
        # collision_admm_cost, whatever data set_params installs later
        self._setup_duals = self.get_state()["y"]

    @property
    def setup_duals(self):
        return self._setup_duals

    # -- iteration ------------------------------------------------------
    def iterate(self, n_iters):
        _check(lib().admm_iterate(self._h, int(n_iters)), "admm_iterate")

    def solve(self, max_iters, check_every=8):
        res = (CadmmResult * self.n_scen)()
        code = lib().admm_solve(self._h, int(max_iters), int(check_every), res)
        _check(code, "admm_solve", allow=(CADMM_OK, CADMM_NOT_CONVERGED))
        return code, [dict(iters=r.iters, converged=bool(r.converged), r_pri=r.r_pri, r_dual=r.r_dual,
                           cost=r.cost, min_alpha=r.min_alpha, unconverged_pairs=r.unconverged_pairs,
                           active_bounds=r.active_bounds)
                      for r in res]

    def reset(self):
        _check(lib().admm_reset(self._h), "admm_reset")

    # -- state ----------------------------------------------------------
    def _state_tensors(self):
        torch = _torch()
        f = dict(dtype=torch.float32, device=self.device)
        return dict(x=torch.empty(self.n_scen, self.N + 1, self.n_s, **f),
                    u=torch.empty(self.n_scen, self.N, self.n_u, **f),
                    y=torch.empty(self.y_floats, **f),
                    zeta=torch.empty(self.n_pairs, **f),
                    xi=torch.empty(self.n_pairs * self.dim, **f))

    def get_state(self):
        st = self._state_tensors()
        _check(lib().admm_get_state(self._h, _ptr(st["x"]), _ptr(st["u"]), _ptr(st["y"]),
                                    _ptr(st["zeta"]), _ptr(st["xi"])), "admm_get_state")
        return st

    def _state_sizes(self):
        return (self.n_scen * (self.N + 1) * self.n_s, self.n_scen * self.N * self.n_u, self.y_floats,
                self.n_pairs, self.n_pairs * self.dim)

    def get_state_host(self):
        """The iterate as FP64 numpy arrays (shapes as get_state), read back
        in one device-to-host copy."""
        torch = _torch()
        sizes = self._state_sizes()
        flat = torch.empty(sum(sizes), dtype=torch.float32, device=self.device)
        views = list(torch.split(flat, sizes))
        _check(lib().admm_get_state(self._h, *[_ptr(v) for v in views]), "admm_get_state")
        host = flat.cpu().numpy().astype(np.float64)
        out, o = {}, 0
        shapes = ((self.n_scen, self.N + 1, self.n_s), (self.n_scen, self.N, self.n_u), (self.y_floats,),
                  (self.n_pairs,), (self.n_pairs * self.dim,))
        for name, n, shp in zip(("x", "u", "y", "zeta", "xi"), sizes, shapes):
            out[name] = host[o:o + n].reshape(shp)
            o += n
        return out

    def set_state(self, x=None, u=None, y=None, zeta=None, xi=None):
        torch = _torch()
        given = (x, u, y, zeta, xi)
        if all(t is None or isinstance(t, np.ndarray) for t in given):
            # host arrays: one host-to-device copy for all parts
            sizes = self._state_sizes()
            arrs = []
            for t, n in zip(given, sizes):
                if t is None:
                    continue
                a = np.ascontiguousarray(t, dtype=np.float32).ravel()
                if a.size != n:
                    raise ValueError(f"state part has {a.size} floats, expected {n}")
                arrs.append(a)
            if not arrs:
                return [None] * 5
            dev = torch.from_numpy(np.concatenate(arrs)).to(self.device)
            views = iter(torch.split(dev, [a.size for a in arrs]))
            parts = [None if t is None else next(views) for t in given]
            _check(lib().admm_set_state(self._h, *[_ptr(p) for p in parts]), "admm_set_state")
            self._keep_set = (dev, parts)   # keep alive until the stream has consumed them
            return parts

        def prep(t, n):
            if t is None:
                return None
            t = torch.as_tensor(t, dtype=torch.float32, device=self.device).contiguous()
            if t.numel() != n:
                raise ValueError(f"state part has {t.numel()} floats, expected {n}")
            return t
        parts = [prep(x, self.n_scen * (self.N + 1) * self.n_s), prep(u, self.n_scen * self.N * self.n_u),
                 prep(y, self.y_floats), prep(zeta, self.n_pairs), prep(xi, self.n_pairs * self.dim)]
        _check(lib().admm_set_state(self._h, *[_ptr(p) for p in parts]), "admm_set_state")
        self._keep_set = parts   # keep alive until the stream has consumed them
        return parts

    def history(self, max_rows):
        rp = np.zeros((max_rows, self.n_scen), np.float32)
        rd = np.zeros((max_rows, self.n_scen), np.float32)
        rows = lib().admm_get_history(self._h, int(max_rows), rp.ctypes.data_as(_vp), rd.ctypes.data_as(_vp))
        if rows < 0:
            raise CadmmError(-rows, "admm_get_history")
        return rp[:rows], rd[:rows]

    def scales(self):
        torch = _torch()
        a = torch.empty(self.n_pairs, dtype=torch.float32, device=self.device)
        _check(lib().admm_scales(self._h, _ptr(a)), "admm_scales")
        return a

    def phase_times(self, n_iters):
        """Mean ms of (pair, trajectory, multiplier, residual) phases over
        n_iters eagerly launched iterations (advances the iterate)."""
        out = (ctypes.c_float * 4)()
        _check(lib().admm_phase_times(self._h, int(n_iters), out), "admm_phase_times")
        return list(out)

    def launch_config(self):
        """(pair blocks per workgroup, workgroups, lanes per pair QP)."""
        w, g, l = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().admm_launch_config(self._h, ctypes.byref(w), ctypes.byref(g), ctypes.byref(l)),
               "admm_launch_config")
        return w.value, g.value, l.value

    # -- differentiation --------------------------------------------------
    def reset_duals(self):
        """Scale-LP certificates at the current trajectory, zero multipliers."""
        _check(lib().admm_reset_duals(self._h), "admm_reset_duals")

    def set_reference(self, x_ref):
        """Replace the reference trajectory [n_scen, N+1, n_s] (FP64 copy)."""
        x = np.ascontiguousarray(_host(x_ref), dtype=np.float64).ravel()
        if x.size != self.n_scen * (self.prob["N"] + 1) * self.n_s:
            raise ValueError(f"x_ref has {x.size} values, expected {self.n_scen * (self.prob['N'] + 1) * self.n_s}")
        _check(lib().admm_set_reference(self._h, x.ctypes.data_as(_dp)), "admm_set_reference")

    def set_params(self, obs_d=None, x0=None):
        """Replace the obstacle offsets d [F_o] and/or initial states x0
        [n_scen, n_s] (anything numpy can read; copied as FP64). The iterate
        is left alone: reset() or record() start from the new data."""
        d = None if obs_d is None else np.ascontiguousarray(_host(obs_d), dtype=np.float64).ravel()
        x = None if x0 is None else np.ascontiguousarray(_host(x0), dtype=np.float64).ravel()
        if d is not None and d.size != len(self.prob["obs_d"]):
            raise ValueError(f"obs_d has {d.size} values, expected {len(self.prob['obs_d'])}")
        if x is not None and x.size != self.n_scen * self.n_s:
            raise ValueError(f"x0 has {x.size} values, expected {self.n_scen * self.n_s}")
        _check(lib().admm_set_params(self._h, None if d is None else d.ctypes.data_as(_dp),
                                     None if x is None else x.ctypes.data_as(_dp)), "admm_set_params")

    def grad_workspace_size(self, n_iters, ckpt_every=10):
        n = ctypes.c_size_t()
        _check(lib().admm_grad_workspace_size(self._h, int(n_iters), int(ckpt_every), ctypes.byref(n)),
               "admm_grad_workspace_size")
        return n.value

    def record(self, n_iters, ckpt_every=10):
        """Run exactly n_iters iterations from s^0 = LQ(x0), zero multipliers
        and the current y, keeping checkpoints for backward(). Returns the
        per-scenario tracking cost of the last iterate (device tensor)."""
        torch = _torch()
        nbytes = self.grad_workspace_size(n_iters, ckpt_every)
        gw = getattr(self, "_grad_ws", None)
        if gw is None or gw.numel() < nbytes + 256:
            self._grad_ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._grad_ws.data_ptr() + 255) & ~255
        cost = torch.empty(self.n_scen, dtype=torch.float32, device=self.device)
        _check(lib().admm_record(self._h, int(n_iters), int(ckpt_every), ctypes.c_void_p(ptr), nbytes, _ptr(cost)),
               "admm_record")
        self._grad_rec = (ptr, nbytes)
        return cost

    def backward(self, scale=1.0):
        """scale * (dL/dd [F_o], dL/dx0 [n_scen, n_s]) of the recorded run,
        L = sum_s F_s(x^K, u^K), y^0 held fixed (device tensors)."""
        torch = _torch()
        rec = getattr(self, "_grad_rec", None)
        if rec is None:
            raise RuntimeError("backward() needs a record() first")
        f = dict(dtype=torch.float32, device=self.device)
        gd = torch.empty(max(len(self.prob["obs_d"]), 1), **f)
        gx = torch.empty(self.n_scen, self.n_s, **f)
        _check(lib().admm_backward(self._h, ctypes.c_void_p(rec[0]), rec[1], float(scale), _ptr(gd), _ptr(gx)),
               "admm_backward")
        return gd[:len(self.prob["obs_d"])], gx

    def close(self):
        if getattr(self, "_h", None):
            lib().collision_admm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def collision_admm_setup(prob, **kw):
    return Handle(prob, **kw)


def _host(a):
    """numpy view of an array or tensor (tensors are copied to the host)."""
    if hasattr(a, "detach"):
        return a.detach().to("cpu").numpy()
    return np.asarray(a)


def _autograd_function():
    torch = _torch()

    class CollisionADMMCost(torch.autograd.Function):
        """L(d, x0; y0) = sum_s F_s(x^K, u^K) after exactly K ADMM iterations
        from s^0 = LQ(x0), zero multipliers and the given initial duals y0,
        which are held fixed (not recomputed from d or x0), with the forward
        run on the GPU (admm_record) and the gradient from the reverse pass
        (admm_backward): value and gradient describe the same map. One
        pending backward per handle: a second forward on the same handle
        replaces the first."""

        @staticmethod
        def forward(ctx, obs_d, x0, handle, n_iters, ckpt_every, y0):
            handle.set_params(obs_d=obs_d, x0=x0)
            handle.reset()                       # s^0 = LQ(x0), zeta = xi = 0
            handle.set_state(y=y0)               # y^0 held fixed
            cost = handle.record(int(n_iters), int(ckpt_every))
            ctx.handle = handle
            ctx.shapes = (obs_d.shape, obs_d.dtype, obs_d.device, x0.shape, x0.dtype, x0.device)
            return cost.sum().to(obs_d.dtype).to(obs_d.device)

        @staticmethod
        def backward(ctx, g):
            ds, dd, ddev, xs, xd, xdev = ctx.shapes
            gd, gx = ctx.handle.backward(float(g))
            return (gd.reshape(ds).to(dtype=dd, device=ddev), gx.reshape(xs).to(dtype=xd, device=xdev),
                    None, None, None, None)

    return CollisionADMMCost


_COST_FN = None


def collision_admm_cost(obs_d, x0, handle, n_iters, ckpt_every=10, y0=None):
    """Differentiable tracking cost after n_iters ADMM iterations (see
    CollisionADMMCost); obs_d and x0 are torch tensors. y0 (canonical dual
    layout) is held fixed; by default the scale-LP certificates the handle
    computed at setup, i.e. at the descriptor's own offsets and initial
    states, whatever obs_d and x0 are passed."""
    global _COST_FN
    if _COST_FN is None:
        _COST_FN = _autograd_function()
    if y0 is None:
        y0 = handle.setup_duals
    return _COST_FN.apply(obs_d, x0, handle, n_iters, ckpt_every, y0)


def pair_qp_batch(row_ptr, K, kappa, yhat, bhat, eps, max_sweeps=0, stream=None, solver=CADMM_PAIR_NEWTON,
                  work=None, noalloc=False):
    """Stateless batch of proximal dual-update QPs (device tensors in, out).

    row_ptr int32 [P+1]; K float32 [rows, dim+1]; kappa, yhat [rows];
    bhat [P, dim+1]. Returns (y [rows], r [P, dim+1], nu [P], status int32 [P]).
    solver: CADMM_PAIR_NEWTON (dual Newton) or CADMM_PAIR_LEMKE (the
    elimination / LCP / Lemke route). work: a device uint8 tensor for the
    dual Newton's two-launch form (pair_qp_batch_workspace_size bytes past a
    256-byte aligned start); noalloc: the library's static buffer instead
    (pair_qp_batch_noalloc)."""
    torch = _torch()
    n_pairs = row_ptr.numel() - 1
    dim = K.shape[1] - 1
    y = torch.empty_like(yhat)
    r = torch.empty_like(bhat)
    nu = torch.empty(n_pairs, dtype=torch.float32, device=K.device)
    status = torch.empty(n_pairs, dtype=torch.int32, device=K.device)
    wptr, wbytes = None, 0
    if work is not None:
        wptr = (work.data_ptr() + 255) & ~255
        wbytes = work.numel() - (wptr - work.data_ptr())
    b = CadmmPairBatch(n_pairs, dim, _ptr(row_ptr), _ptr(K), _ptr(kappa), _ptr(yhat), _ptr(bhat),
                       float(eps), int(max_sweeps), _ptr(y), _ptr(r), _ptr(nu), _ptr(status), int(solver),
                       wptr, int(wbytes))
    fn = lib().pair_qp_batch_noalloc if noalloc else lib().pair_qp_batch
    _check(fn(ctypes.byref(b), _stream_ptr(stream)), "pair_qp_batch_noalloc" if noalloc else "pair_qp_batch")
    return y, r, nu, status


def model_step(model, model_par, s, u):
    """One host step s + dt f_c(s, u) of a built-in nonlinear model (FP64)."""
    par = np.zeros(8)
    par[:len(model_par)] = model_par
    s = np.ascontiguousarray(s, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(s)
    _check(lib().cadmm_model_step(int(model), par.ctypes.data_as(_dp), s.ctypes.data_as(_dp), u.ctypes.data_as(_dp),
                                  out.ctypes.data_as(_dp)), "cadmm_model_step")
    return out


def pair_qp_batch_workspace_size(n_pairs):
    n = ctypes.c_size_t()
    _check(lib().pair_qp_batch_workspace_size(int(n_pairs), ctypes.byref(n)), "pair_qp_batch_workspace_size")
    return n.value


def pair_scale_batch(a_ptr, A, b, o_ptr, Cp, dp, stream=None):
    """Stateless batch of scale LPs in the part frame (device tensors).

    Returns (alpha [P], lam [rows of A], mu [rows of Cp], status [P])."""
    torch = _torch()
    n_pairs = a_ptr.numel() - 1
    dim = A.shape[1]
    alpha = torch.empty(n_pairs, dtype=torch.float32, device=A.device)
    lam = torch.empty(A.shape[0], dtype=torch.float32, device=A.device)
    mu = torch.empty(Cp.shape[0], dtype=torch.float32, device=A.device)
    status = torch.empty(n_pairs, dtype=torch.int32, device=A.device)
    sb = CadmmScaleBatch(n_pairs, dim, _ptr(a_ptr), _ptr(A), _ptr(b), _ptr(o_ptr), _ptr(Cp), _ptr(dp),
                         _ptr(alpha), _ptr(lam), _ptr(mu), _ptr(status))
    _check(lib().pair_scale_batch(ctypes.byref(sb), _stream_ptr(stream)), "pair_scale_batch")
    return alpha, lam, mu, status
