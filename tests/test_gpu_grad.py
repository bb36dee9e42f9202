"""GPU reverse pass (admm_record / admm_backward and the autograd Function)
against the FP64 oracle's reverse pass through the same unrolled iteration.

The differentiated map is L(d, x0) = sum_s F_s(x^K, u^K) after exactly K
iterations (Sec. IV-B, no stopping test) from s^0 = LQ(x0), zero multipliers
and a fixed y^0 (Sec. IV-A eq. navigation_cost for F). y^0 is the oracle's
scale-LP certificate at s^0 scaled by 1.01 (a generic, non fixed-point dual,
as in the oracle's own finite-difference pins), given to both sides.

Two comparisons, each with a fixed bar:
- The reverse pass alone: the oracle's FP64 reverse recursion is run at the
  GPU's own forward iterates (read back after every iteration; they are
  bitwise those admm_record keeps), so the comparison sees only the FP32
  arithmetic of the reverse kernels. Bar: 1e-4 relative for the offset
  gradient (measured <= 1e-5); 1e-3 for the x0 gradient, whose cotangent
  sum_t (A^T)^t (xbar_t - H_t w_t) over each trajectory QP cancels terms of
  the size of its seeds in FP32 (measured 1.1e-5 to 6.4e-4).
- End to end: against the oracle's gradient through its own FP64 forward run.
  The cost seeds 2 Q_s (x^K - x_ref) of the reverse pass then carry the FP32
  forward trajectory error divided by the tracking error, which is small
  next to the positions of the scene (kappa = ||x^K|| / ||x^K - x_ref|| is
  1.6e2 to 5e3 here). Bar: 2e-2 relative (a fixed bar; measured values are
  printed).
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2406_07048_amd as cadmm  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_REVERSE = 1e-4
TOL_REVERSE_X0 = 1e-3
TOL_END_TO_END = 2e-2


def _y0(p):
    return oracle.Problem(p).init_state()["y"] * 1.01


def _oracle_xK(p, K, y0):
    q = dict(p)
    q["eps_pri"] = -1.0
    q["eps_dual"] = -1.0
    P = oracle.Problem(q)
    st = P.init_state()
    st["y"][:] = y0
    P.run(st, K)
    return st["x"]


def _gpu(h, K, every, y0):
    h.set_state(y=torch.as_tensor(y0, dtype=torch.float32))
    cost = h.record(K, every)
    st = h.get_state()
    gd, gx = h.backward(1.0)
    torch.cuda.synchronize()
    return (float(cost.double().sum()), gd.cpu().numpy().astype(np.float64), gx.cpu().numpy().astype(np.float64),
            {k: v.cpu().numpy() for k, v in st.items()})


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _no_stop(p):
    q = dict(p)
    q["eps_pri"] = -1.0
    q["eps_dual"] = -1.0
    return q


def _gpu_iterates(h, K, y0):
    """The GPU's forward iterates k = 0..K from s^0, zero multipliers and y0
    (one graph replay per iteration; the stopping test is off)."""
    h.reset()
    h.set_state(y=torch.as_tensor(y0, dtype=torch.float32))
    its = []
    for k in range(K + 1):
        if k:
            h.iterate(1)
        st = h.get_state()
        torch.cuda.synchronize()
        its.append({a: v.double().cpu().numpy() for a, v in st.items()})
    return its


@pytest.mark.parametrize("name,K,every", [("c1", 1, 1), ("c1", 10, 3), ("c3", 10, 4), ("c3", 100, 10)])
def test_reverse_pass_at_the_gpu_iterates(name, K, every):
    """admm_backward against the oracle's reverse pass at the GPU's own
    forward iterates (fixed bar TOL_REVERSE)."""
    print(f"[grad reverse] {name} K={K} every={every}", flush=True)
    p = _no_stop(workloads.make(name))
    y0 = _y0(p)
    h = cadmm.Handle(p)
    Lg, gdg, gxg, st = _gpu(h, K, every, y0)
    its = _gpu_iterates(h, K, y0)
    h.close()
    for a in ("x", "u", "y", "zeta", "xi"):      # the recorded run is the one read back
        assert np.array_equal(its[-1][a].ravel(), st[a].astype(np.float64).ravel()), a
    Lo, gdo, gxo = oracle.grad_at_iterates(p, its)
    ed, ex = _rel(gdg, gdo), _rel(gxg, gxo)
    print(f"  L rel {abs(Lg - Lo) / Lo:.2e} grad_d rel {ed:.2e} grad_x0 rel {ex:.2e}")
    assert abs(Lg - Lo) <= 1e-5 * abs(Lo)
    assert ed <= TOL_REVERSE
    assert ex <= TOL_REVERSE_X0


@pytest.mark.parametrize("name,K,every", [("c1", 10, 3), ("c3", 10, 4), ("c3", 100, 10)])
def test_gradient_matches_oracle_end_to_end(name, K, every):
    """The GPU gradient (FP32 forward and reverse) against the oracle's FP64
    forward and reverse passes (fixed bar TOL_END_TO_END)."""
    print(f"[grad end to end] {name} K={K} every={every}", flush=True)
    p = workloads.make(name)
    y0 = _y0(p)
    Lo, gdo, gxo = oracle.grad_fixed_y0(p, K, y0)
    xo = _oracle_xK(p, K, y0)
    h = cadmm.Handle(p)
    Lg, gdg, gxg, st = _gpu(h, K, every, y0)
    h.close()
    e_x = _rel(st["x"], xo)
    kappa = np.linalg.norm(xo[:, 1:]) / np.linalg.norm((xo - p["x_ref"])[:, 1:])
    ed, ex = _rel(gdg, gdo), _rel(gxg, gxo)
    print(f"  e_x {e_x:.2e} kappa {kappa:.2e} L rel {abs(Lg - Lo) / Lo:.2e} grad_d rel {ed:.2e} grad_x0 rel {ex:.2e}")
    assert e_x <= 1e-4
    assert abs(Lg - Lo) <= TOL_END_TO_END * abs(Lo)
    assert ed <= TOL_END_TO_END
    assert ex <= TOL_END_TO_END


@pytest.mark.parametrize("name,K,everies", [("c1", 10, (1, 4, 10)), ("c3", 8, (1, 3, 8))])
def test_checkpoint_interval_does_not_change_the_gradient(name, K, everies):
    """The replay of a segment from its checkpoint repeats the recorded run
    bit for bit, so the gradient is bitwise independent of the interval."""
    print(f"[grad-ckpt] {name} K={K} every={everies}", flush=True)
    p = workloads.make(name)
    y0 = _y0(p)
    h = cadmm.Handle(p)
    outs = [_gpu(h, K, e, y0) for e in everies]
    h.close()
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2])
        assert o[0] == outs[0][0]


def test_backward_leaves_the_last_iterate():
    """After admm_backward the handle holds iterate K, as after admm_record."""
    p = workloads.make("c1")
    h = cadmm.Handle(p)
    h.reset()
    h.record(7, 3)
    a = {k: v.cpu().numpy() for k, v in h.get_state().items()}
    h.backward()
    b = {k: v.cpu().numpy() for k, v in h.get_state().items()}
    h.close()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_autograd_function_matches_backward():
    """collision_admm_cost: the value is the recorded cost, and torch.autograd
    gives admm_backward scaled by the upstream gradient (2 here, exact)."""
    p = workloads.make("c1")
    h = cadmm.Handle(p)
    d = torch.tensor(p["obs_d"], dtype=torch.float64, requires_grad=True)
    x0 = torch.tensor(p["x0"], dtype=torch.float64, requires_grad=True)
    L = cadmm.collision_admm_cost(d, x0, h, 10, 4)
    gd, gx = torch.autograd.grad(2.0 * L, (d, x0))
    h.reset()
    cost = h.record(10, 4)
    gd1, gx1 = h.backward(1.0)
    torch.cuda.synchronize()
    assert float(L.detach()) == pytest.approx(float(cost.sum()), rel=1e-6)
    assert torch.equal(gd.float().cpu(), 2 * gd1.cpu())
    assert torch.equal(gx.float().cpu(), 2 * gx1.cpu().reshape(gx.shape))
    h.close()


def test_autograd_function_holds_y0_fixed():
    """At moved offsets and initial states the Function's value is the
    oracle's map L(d, x0; y0) with the setup's y0 (not the certificates of the
    moved data), and its gradient is the oracle's gradient of that same map:
    value and gradient describe one function, the one whose gradient the
    oracle's central-difference pins check."""
    p = workloads.make("c1")
    K = 8
    rng = np.random.default_rng(7)
    q = dict(p)
    q["obs_d"] = p["obs_d"] + 0.05 * rng.normal(size=p["obs_d"].shape)
    q["x0"] = p["x0"] + 0.02 * rng.normal(size=p["x0"].shape)
    y0 = oracle.Problem(p).init_state()["y"]          # the certificates at p, as setup computed them
    assert not np.allclose(oracle.Problem(q).init_state()["y"], y0)
    h = cadmm.Handle(p)
    d = torch.tensor(q["obs_d"], dtype=torch.float64, requires_grad=True)
    x0 = torch.tensor(q["x0"], dtype=torch.float64, requires_grad=True)
    L = cadmm.collision_admm_cost(d, x0, h, K, 3)
    gd, gx = torch.autograd.grad(L, (d, x0))
    h.close()
    Lo = oracle.loss_fixed_y0(q, K, y0)
    Lo2, gdo, gxo = oracle.grad_fixed_y0(q, K, y0)
    assert Lo2 == pytest.approx(Lo, rel=1e-12)
    print(f"  L rel {abs(float(L) - Lo) / Lo:.2e} grad_d rel {_rel(gd.numpy(), gdo):.2e} "
          f"grad_x0 rel {_rel(gx.numpy(), gxo):.2e}")
    assert abs(float(L) - Lo) <= 1e-5 * Lo
    assert _rel(gd.numpy(), gdo) <= TOL_END_TO_END
    assert _rel(gx.numpy(), gxo) <= TOL_END_TO_END


def test_set_params_moves_the_gradient_like_the_oracle():
    """New offsets and initial states through admm_set_params: the GPU
    gradient follows the oracle's at the perturbed data."""
    p = workloads.make("c1")
    rng = np.random.default_rng(3)
    q = dict(p)
    q["obs_d"] = p["obs_d"] + 0.05 * rng.normal(size=p["obs_d"].shape)
    q["x0"] = p["x0"] + 0.02 * rng.normal(size=p["x0"].shape)
    y0 = _y0(q)
    Lo, gdo, gxo = oracle.grad_fixed_y0(q, 10, y0)
    h = cadmm.Handle(p)
    h.set_params(obs_d=q["obs_d"], x0=q["x0"])
    Lg, gdg, gxg, st = _gpu(h, 10, 5, y0)
    h.close()
    xo = _oracle_xK(q, 10, y0)
    assert _rel(st["x"], xo) <= 1e-4
    assert _rel(gdg, gdo) <= TOL_END_TO_END
    assert _rel(gxg, gxo) <= TOL_END_TO_END


def test_no_obstacles_gives_the_lq_gradient():
    """Without obstacles L is the LQ tracking cost of x0 alone; the offsets
    have no gradient and the x0 gradient matches the oracle's."""
    p = workloads.with_obstacles(workloads.make("c1"), [[]])
    p["x0"] = p["x0"] + np.array([[0.5, -0.4, 0.05, 0.3]])   # off the reference: L > 0
    Lo, gdo, gxo = oracle.grad_fixed_y0(p, 3, np.zeros(0))
    assert Lo > 1e-3 and np.linalg.norm(gxo) > 1e-3
    h = cadmm.Handle(p)
    h.reset()
    cost = h.record(3, 2)
    gd, gx = h.backward()
    torch.cuda.synchronize()
    h.close()
    assert gd.numel() == 0
    assert float(cost.sum()) == pytest.approx(Lo, rel=1e-5)
    assert _rel(gx.cpu().numpy(), gxo) <= TOL_REVERSE_X0


def test_invalid_reverse_calls():
    """Error paths of the ABI: backward with nothing recorded (checked
    before any device work), zero iterations, zero checkpoint interval."""
    import ctypes
    p = workloads.make("c1")
    h = cadmm.Handle(p)
    assert cadmm.lib().admm_backward(h._h, ctypes.c_void_p(256), 1 << 20, 1.0, None, None) == cadmm.CADMM_INVALID
    with pytest.raises(RuntimeError):
        h.backward()                      # the binding refuses too
    with pytest.raises(cadmm.CadmmError):
        h.grad_workspace_size(0, 1)
    with pytest.raises(cadmm.CadmmError):
        h.record(5, 0)
    h.close()
