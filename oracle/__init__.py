"""FP64 CPU oracle for the ADMM collision-avoidance path (arXiv 2406.07048).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path. It shares no code
with the HIP library; both sides only share the seeded generator in
``workloads``.

The arithmetic lives in ``cadmm_oracle.c`` (plain C, double precision); this
module builds it with gcc and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cadmm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_cadmm_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle shared library (gcc, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_up = ctypes.POINTER(ctypes.c_ubyte)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n_s", ctypes.c_int), ("n_u", ctypes.c_int), ("N", ctypes.c_int),
        ("n_parts", ctypes.c_int), ("n_scen", ctypes.c_int),
        ("part_face_ptr", _ip), ("part_A", _dp), ("part_b", _dp), ("part_off", _dp),
        ("obs_ptr", _ip), ("obs_face_ptr", _ip), ("obs_C", _dp), ("obs_d", _dp),
        ("A_dyn", _dp), ("B_dyn", _dp), ("c_dyn", _dp),
        ("pos_idx", _ip), ("att_idx", _ip), ("att_kind", ctypes.c_int),
        ("Q_s", _dp), ("Q_u", _dp), ("x_ref", _dp), ("x0", _dp),
        ("sigma", ctypes.c_double), ("eps_prox", ctypes.c_double),
        ("eps_pri", ctypes.c_double), ("eps_dual", ctypes.c_double),
        ("dyn_ts", ctypes.c_int), ("dyn_ss", ctypes.c_int), ("model", ctypes.c_int),
        ("model_par", ctypes.c_double * 8),
        ("s_lo", _dp), ("s_hi", _dp), ("u_lo", _dp), ("u_hi", _dp),
    ]


def _declare(L):
    L.orc_scale_lp.restype = ctypes.c_int
    L.orc_scale_lp.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp,
                               _dp, _dp, _dp, _dp, _dp]
    L.orc_pair_qp.restype = ctypes.c_int
    L.orc_pair_qp.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp,
                              ctypes.c_double, _dp, _dp, ctypes.c_double, _dp]
    L.orc_pair_qp_lemke.restype = ctypes.c_int
    L.orc_pair_qp_lemke.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp,
                                    ctypes.c_double, _dp, _dp, ctypes.c_double, _dp]
    L.orc_traj_qp.restype = ctypes.c_int
    L.orc_traj_qp.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp,
                              _dp, _dp, _dp, _dp, _dp]
    L.orc_traj_qp_bounded.restype = ctypes.c_int
    L.orc_traj_qp_bounded.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp,
                                      _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _ip]
    PP = ctypes.POINTER(_Problem)
    L.orc_y_size.restype = ctypes.c_long
    L.orc_y_size.argtypes = [PP]
    L.orc_admm_init.restype = ctypes.c_int
    L.orc_admm_init.argtypes = [PP, _dp, _dp, _dp, _dp, _dp]
    L.orc_scale_all.restype = ctypes.c_int
    L.orc_scale_all.argtypes = [PP, _dp, _dp, _dp]
    L.orc_pair_phase.restype = ctypes.c_int
    L.orc_pair_phase.argtypes = [PP, _dp, _dp, _dp, _dp, _up, _dp]
    L.orc_traj_phase.restype = ctypes.c_int
    L.orc_traj_phase.argtypes = [PP, _dp, _dp, _dp, _dp, _up, _dp, _dp]
    L.orc_mult_phase.restype = None
    L.orc_mult_phase.argtypes = [PP, _dp, _dp, _up, _dp, _dp, _dp]
    L.orc_cost.restype = ctypes.c_double
    L.orc_cost.argtypes = [PP, ctypes.c_int, _dp, _dp]
    L.orc_admm_run.restype = ctypes.c_int
    L.orc_admm_run.argtypes = [PP, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _ip]
    L.orc_admm_grad.restype = ctypes.c_int
    L.orc_admm_grad.argtypes = [PP, ctypes.c_int, _dp, _dp, _dp, _dp]
    L.orc_admm_grad_at.restype = ctypes.c_int
    L.orc_admm_grad_at.argtypes = [PP, ctypes.c_int] + [_dp] * 5 + [_dp, _dp, _dp]
    L.orc_pairqp_vjp.restype = ctypes.c_int
    L.orc_pairqp_vjp.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp, ctypes.c_double,
                                 _dp, _dp, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_traj_vjp.restype = ctypes.c_int
    L.orc_traj_vjp.argtypes = [PP] + [_dp] * 12
    L.orc_model_step.restype = ctypes.c_int
    L.orc_model_step.argtypes = [PP, _dp, _dp, _dp, _dp, _dp]
    L.orc_set_threads.restype = ctypes.c_int
    L.orc_set_threads.argtypes = [ctypes.c_int]


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(n):
    """Set the OpenMP thread count; returns the count now in effect."""
    return lib().orc_set_threads(int(n))


# ---------------------------------------------------------------- single pair
def scale_lp(A, b, Cp, dp):
    """Scale LP (Sec. III-A) of one part/obstacle pair in the part frame.

    Returns (alpha, x, lam, mu, gap, status)."""
    A, b, Cp, dp = _f64(A), _f64(b), _f64(Cp), _f64(dp)
    dim = A.shape[1]
    alpha = np.zeros(1)
    x = np.zeros(dim)
    lam = np.zeros(len(b))
    mu = np.zeros(len(dp))
    gap = np.zeros(1)
    st = lib().orc_scale_lp(dim, len(b), _d(A), _d(b), len(dp), _d(Cp), _d(dp),
                            _d(alpha), _d(x), _d(lam), _d(mu), _d(gap))
    return float(alpha[0]), x, lam, mu, float(gap[0]), st


def pair_qp(A, b, Cp, dp, zeta, xi, yhat, eps):
    """Dual-update sub-problem (Sec. IV-C) with the Jacobi-scaled proximal term.

    Returns (y, iterations) ; iterations < 0 means failure."""
    A, b, Cp, dp = _f64(A), _f64(b), _f64(Cp), _f64(dp)
    xi, yhat = _f64(xi), _f64(yhat)
    dim = A.shape[1]
    y = np.zeros(len(b) + len(dp) + 1)
    it = lib().orc_pair_qp(dim, len(b), _d(A), _d(b), len(dp), _d(Cp), _d(dp),
                           float(zeta), _d(xi), _d(yhat), float(eps), _d(y))
    return y, it


def pair_qp_lemke(A, b, Cp, dp, zeta, xi, yhat, eps):
    """The dual-update sub-problem solved the paper's way (Sec. IV-C): the
    equality eliminated, the KKT conditions as an LCP, Lemke's method.

    Returns (y, status); status 0 = solved."""
    A, b, Cp, dp = _f64(A), _f64(b), _f64(Cp), _f64(dp)
    xi, yhat = _f64(xi), _f64(yhat)
    dim = A.shape[1]
    y = np.zeros(len(b) + len(dp) + 1)
    st = lib().orc_pair_qp_lemke(dim, len(b), _d(A), _d(b), len(dp), _d(Cp), _d(dp),
                                 float(zeta), _d(xi), _d(yhat), float(eps), _d(y))
    return y, st


def traj_qp(A, B, c, x0, H, h, Q_u):
    """LQ problem with stage terms (H_t, h_t), t = 1..N, and input cost u^T Q_u u.
    A, B, c are one model ([n_s, n_s], [n_s, n_u], [n_s]) or one per step
    ([N, n_s, n_s], [N, n_s, n_u], [N, n_s])."""
    A, B, c, x0, H, h, Q_u = map(_f64, (A, B, c, x0, H, h, Q_u))
    n_s, n_u = B.shape[-2:]
    N = H.shape[0]
    ts = 1 if A.ndim == 3 else 0
    x = np.zeros((N + 1, n_s))
    u = np.zeros((N, n_u))
    st = lib().orc_traj_qp(n_s, n_u, N, _d(A), _d(B), _d(c), ts, _d(x0), _d(H), _d(h), _d(Q_u),
                           _d(x), _d(u))
    if st:
        raise RuntimeError("oracle trajectory QP: Hessian not positive definite")
    return x, u


def traj_qp_bounded(A, B, c, x0, H, h, Q_u, s_lo=None, s_hi=None, u_lo=None, u_hi=None):
    """traj_qp with the bounds s_lo <= x_t <= s_hi (t = 1..N) and
    u_lo <= u_t <= u_hi (t = 0..N-1); None or infinite entries: no bound.
    Returns (x, u, n_active)."""
    A, B, c, x0, H, h, Q_u = map(_f64, (A, B, c, x0, H, h, Q_u))
    n_s, n_u = B.shape[-2:]
    N = H.shape[0]
    ts = 1 if A.ndim == 3 else 0
    lims = [None if v is None else _f64(v) for v in (s_lo, s_hi, u_lo, u_hi)]
    x = np.zeros((N + 1, n_s))
    u = np.zeros((N, n_u))
    na = ctypes.c_int()
    st = lib().orc_traj_qp_bounded(n_s, n_u, N, _d(A), _d(B), _d(c), ts, _d(x0), _d(H), _d(h), _d(Q_u),
                                   *[None if v is None else _d(v) for v in lims], _d(x), _d(u), ctypes.byref(na))
    if st:
        raise RuntimeError(f"oracle bounded trajectory QP failed (status {st})")
    return x, u, na.value


# ---------------------------------------------------------------- full problem
class Problem:
    """Holds contiguous copies of a workloads problem dict and its C mirror."""

    def __init__(self, prob):
        self.p = prob
        self._keep = {}
        k = self._keep
        for name in ("part_A", "part_b", "part_off", "obs_C", "obs_d", "A_dyn", "B_dyn", "c_dyn",
                     "Q_s", "Q_u", "x_ref", "x0"):
            k[name] = _f64(prob[name])
        for name in ("part_face_ptr", "obs_ptr", "obs_face_ptr", "pos_idx", "att_idx"):
            k[name] = _i32(prob[name])
        st = _Problem()
        st.dim = int(prob["dim"])
        st.n_s = int(prob["n_s"])
        st.n_u = int(prob["n_u"])
        st.N = int(prob["N"])
        st.n_parts = len(prob["part_face_ptr"]) - 1
        st.n_scen = len(prob["obs_ptr"]) - 1
        for name in ("part_A", "part_b", "part_off", "obs_C", "obs_d", "A_dyn", "B_dyn", "c_dyn",
                     "Q_s", "Q_u", "x_ref", "x0"):
            setattr(st, name, _d(k[name]))
        for name in ("part_face_ptr", "obs_ptr", "obs_face_ptr", "pos_idx", "att_idx"):
            setattr(st, name, _i(k[name]))
        st.att_kind = int(prob["att_kind"])
        st.sigma = float(prob["sigma"])
        st.eps_prox = float(prob["eps_prox"])
        st.eps_pri = float(prob["eps_pri"])
        st.eps_dual = float(prob["eps_dual"])
        st.dyn_ts = int(prob.get("dyn_ts", 0))
        st.dyn_ss = int(prob.get("dyn_ss", 0))
        st.model = int(prob.get("model", 0))
        for i, v in enumerate(prob.get("model_par", ())):
            st.model_par[i] = float(v)
        for key, field in (("s_min", "s_lo"), ("s_max", "s_hi"), ("u_min", "u_lo"), ("u_max", "u_hi")):
            if prob.get(key) is not None:
                k[key] = _f64(prob[key])
                setattr(st, field, _d(k[key]))
        self.st = st
        self.ref = ctypes.byref(st)
        self.n_scen = st.n_scen
        self.n_blocks = st.n_parts * int(prob["obs_ptr"][-1])
        self.y_size = int(lib().orc_y_size(self.ref))

    def new_state(self):
        S, N, n_s, n_u, dim = self.n_scen, self.st.N, self.st.n_s, self.st.n_u, self.st.dim
        return dict(x=np.zeros((S, N + 1, n_s)), u=np.zeros((S, N, n_u)),
                    y=np.zeros(self.y_size), zeta=np.zeros(self.n_blocks * N),
                    xi=np.zeros(self.n_blocks * dim * N))

    def init_state(self):
        """s^0 = obstacle-free LQ, zeta = xi = 0, y^0 = scale-LP certificates."""
        s = self.new_state()
        bad = lib().orc_admm_init(self.ref, _d(s["x"]), _d(s["u"]), _d(s["y"]), _d(s["zeta"]), _d(s["xi"]))
        if bad:
            raise RuntimeError("oracle init: scale LP failed")
        return s

    def scale_all(self, x, with_y=False):
        """alpha* of every pair at trajectory x; with_y: also the LP
        certificates (lam*, mu*, max(alpha* - 1, 0)) in the layout of y."""
        N = self.st.N
        alpha = np.zeros(self.n_blocks * N)
        y = np.zeros(self.y_size) if with_y else None
        bad = lib().orc_scale_all(self.ref, _d(_f64(x)), _d(alpha), _d(y) if with_y else None)
        if bad:
            raise RuntimeError("oracle scale LP failed")
        return (alpha, y) if with_y else alpha

    def pair_phase(self, state, active=None):
        y_out = state["y"].copy()
        act = None if active is None else np.ascontiguousarray(active, np.uint8)
        bad = lib().orc_pair_phase(self.ref, _d(state["x"]), _d(state["y"]), _d(state["zeta"]),
                                   _d(state["xi"]), None if act is None else act.ctypes.data_as(_up),
                                   _d(y_out))
        if bad:
            raise RuntimeError(f"oracle pair phase: {bad} failed pair QPs")
        return y_out

    def traj_phase(self, state, y_new, active=None):
        x_out = np.zeros_like(state["x"])
        u_out = state["u"].copy()
        act = None if active is None else np.ascontiguousarray(active, np.uint8)
        bad = lib().orc_traj_phase(self.ref, _d(state["x"]), _d(_f64(y_new)), _d(state["zeta"]),
                                   _d(state["xi"]), None if act is None else act.ctypes.data_as(_up),
                                   _d(x_out), _d(u_out))
        if bad:
            raise RuntimeError("oracle trajectory phase failed")
        return x_out, u_out

    def mult_phase(self, x, y, zeta, xi):
        zeta = zeta.copy()
        xi = xi.copy()
        rpri = np.zeros(self.n_scen)
        lib().orc_mult_phase(self.ref, _d(_f64(x)), _d(_f64(y)), None, _d(zeta), _d(xi), _d(rpri))
        return zeta, xi, rpri

    def traj_vjp(self, state, y_new, xbar, ubar):
        """Adjoints of (y^{k+1}, zeta^k, xi^k, x^k, obstacle offsets, x0) of the
        trajectory phase for cotangents (xbar, ubar) of (x^{k+1}, u^{k+1})."""
        out = dict(y=np.zeros(self.y_size), zeta=np.zeros_like(state["zeta"]), xi=np.zeros_like(state["xi"]),
                   x=np.zeros_like(state["x"]), d=np.zeros(len(self.p["obs_d"])), x0=np.zeros_like(self.p["x0"]))
        bad = lib().orc_traj_vjp(self.ref, _d(state["x"]), _d(_f64(y_new)), _d(state["zeta"]), _d(state["xi"]),
                                 _d(_f64(xbar)), _d(_f64(ubar)), _d(out["y"]), _d(out["zeta"]), _d(out["xi"]),
                                 _d(out["x"]), _d(out["d"]), _d(out["x0"]))
        if bad:
            raise RuntimeError("trajectory VJP failed")
        return out

    def model_step(self, s, u):
        """(F(s, u), dF/ds, dF/du) of the problem's nonlinear model."""
        n_s, n_u = self.st.n_s, self.st.n_u
        F = np.zeros(n_s)
        A = np.zeros((n_s, n_s))
        B = np.zeros((n_s, n_u))
        if lib().orc_model_step(self.ref, _d(_f64(s)), _d(_f64(u)), _d(F), _d(A), _d(B)):
            raise ValueError("the problem has no nonlinear model")
        return F, A, B

    def cost(self, x, u, s=0):
        return lib().orc_cost(self.ref, int(s), _d(_f64(x)), _d(_f64(u)))

    def run(self, state, max_iters):
        """ADMM iterations in place on state; returns history dict."""
        S = self.n_scen
        hp = np.zeros((max_iters, S))
        hd = np.zeros((max_iters, S))
        hc = np.zeros((max_iters, S))
        iters = np.zeros(S, np.int32)
        bad = lib().orc_admm_run(self.ref, int(max_iters), _d(state["x"]), _d(state["u"]), _d(state["y"]),
                                 _d(state["zeta"]), _d(state["xi"]), _d(hp), _d(hd), _d(hc), _i(iters))
        if bad:
            raise RuntimeError(f"oracle ADMM: {bad} failed sub-solves")
        return dict(r_pri=hp, r_dual=hd, cost=hc, iters=iters)


# ---------------------------------------------------------------- gradient
def loss_fixed_y0(prob, K, y0):
    """L = sum_s F_s(x^K, u^K) after exactly K iterations from s^0 = LQ(x0),
    the given y0 and zero multipliers (no early stop)."""
    q = dict(prob)
    q["eps_pri"] = -1.0
    q["eps_dual"] = -1.0
    P = Problem(q)
    st = P.init_state()
    st["y"][:] = y0
    P.run(st, K)
    return sum(P.cost(st["x"], st["u"], s) for s in range(P.n_scen))


def grad_fixed_y0(prob, K, y0):
    """(L, dL/d obstacle offsets [F_o], dL/d x0 [n_scen, n_s]) by the oracle's
    reverse pass through the K unrolled iterations (y0 held fixed)."""
    P = Problem(prob)
    L = np.zeros(1)
    gd = np.zeros(len(prob["obs_d"]))
    gx = np.zeros((P.n_scen, int(prob["n_s"])))
    y0 = _f64(y0)
    bad = lib().orc_admm_grad(P.ref, int(K), _d(y0), _d(L), _d(gd), _d(gx))
    if bad:
        raise RuntimeError(f"oracle gradient: {bad} failed solves")
    return float(L[0]), gd, gx


def grad_at_iterates(prob, iterates):
    """(L, dL/dd, dL/dx0) by the oracle's reverse pass at given iterates:
    ``iterates`` is a list of K + 1 state dicts (x, u, y, zeta, xi), k = 0..K,
    for example another implementation's forward run. The reverse arithmetic
    is that of grad_fixed_y0; only the forward iterates are supplied."""
    P = Problem(prob)
    K = len(iterates) - 1
    cat = {k: _f64(np.stack([np.asarray(it[k], np.float64).ravel() for it in iterates]))
           for k in ("x", "u", "y", "zeta", "xi")}
    L = np.zeros(1)
    gd = np.zeros(len(prob["obs_d"]))
    gx = np.zeros((P.n_scen, int(prob["n_s"])))
    bad = lib().orc_admm_grad_at(P.ref, K, _d(cat["x"]), _d(cat["u"]), _d(cat["y"]), _d(cat["zeta"]),
                                 _d(cat["xi"]), _d(L), _d(gd), _d(gx))
    if bad:
        raise RuntimeError(f"oracle reverse pass: {bad} failed solves")
    return float(L[0]), gd, gx


def pair_qp_vjp(A, b, Cp, dp, zeta, xi, yhat, eps, ybar):
    """Adjoints (dp, Cp, zeta, xi, yhat) of one pair QP for the cotangent ybar."""
    A, b, Cp, dp, xi, yhat, ybar = map(_f64, (A, b, Cp, dp, xi, yhat, ybar))
    dim = A.shape[1]
    dpb = np.zeros(len(dp)); Cpb = np.zeros_like(Cp); zb = np.zeros(1); xib = np.zeros(dim)
    yhb = np.zeros(len(yhat))
    st = lib().orc_pairqp_vjp(dim, len(b), _d(A), _d(b), len(dp), _d(Cp), _d(dp), float(zeta), _d(xi), _d(yhat),
                              float(eps), _d(ybar), _d(dpb), _d(Cpb), _d(zb), _d(xib), _d(yhb))
    if st:
        raise RuntimeError("pair QP VJP failed")
    return dpb, Cpb, float(zb[0]), xib, yhb
