"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, and rejects invalid descriptors."""
import os
import re

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "cadmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char\s*\*|const char\s*\*)\s*\**\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import paper_2406_07048_amd as cadmm
    L = cadmm.lib()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(cadmm._SIGNATURES), "binding and header disagree"


def test_strerror():
    import paper_2406_07048_amd as cadmm
    L = cadmm.lib()
    for code in range(5):
        assert len(L.cadmm_strerror(code)) > 0


def _size_code(prob):
    import paper_2406_07048_amd as cadmm
    try:
        cadmm.cadmm_workspace_size(prob)
        return 0
    except cadmm.CadmmError as e:
        return e.code


def test_workspace_size_counts():
    import paper_2406_07048_amd as cadmm
    p = workloads.make("c2")
    nbytes, nb, npairs, yf = cadmm.cadmm_workspace_size(p)
    assert nb == 2 * 40 and npairs == 2 * 40 * 50
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(p)
    assert yf == tot
    assert nbytes > 4 * (yf + npairs * 3)


@pytest.mark.parametrize("mutate", [
    lambda p: p.__setitem__("part_b", -p["part_b"]),                      # b_i <= 0
    lambda p: p["obs_d"].__setitem__(0, np.nan),                          # non-finite
    lambda p: p["obs_C"].__setitem__(0, np.zeros(p["dim"])),              # zero normal
    lambda p: p.__setitem__("N", 65),                                    # horizon limit
    lambda p: p.__setitem__("sigma", 0.0),
    lambda p: p.__setitem__("eps_prox", -1.0),
    lambda p: p.__setitem__("att_kind", 1),                               # wrong attitude for 2D
    lambda p: p.__setitem__("pos_idx", np.array([0, 9], np.int32)),
])
def test_invalid_descriptors_rejected(mutate):
    p = workloads.make("c1")
    p = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    mutate(p)
    if p["N"] == 65:
        p["x_ref"] = np.zeros((1, 66, 4))
    assert _size_code(p) == 1


def test_too_many_faces_rejected():
    p = workloads.make("c1")
    # one obstacle with 40 faces (limit 32)
    ang = np.linspace(0, 2 * np.pi, 40, endpoint=False)
    C = np.stack([np.cos(ang), np.sin(ang)], 1)
    d = np.full(40, 1.0) + C @ np.array([20.0, 20.0])
    q = workloads.with_obstacles(p, [[(C, d)]])
    assert _size_code(q) == 1


def test_time_varying_and_nonlinear_models_accepted():
    """Per-scenario-and-step models and the nonlinear bicycle / quadrotor
    pass validation; the workspace grows by the uploaded models."""
    import paper_2406_07048_amd as cadmm
    for name in ("c2tv", "c2sqp", "c3sqp"):
        assert _size_code(workloads.make(name)) == 0
    p = workloads.make("c2tv")
    n_tv = cadmm.cadmm_workspace_size(p)[0]
    q = dict(p)
    q.update(A_dyn=p["A_dyn"][0], B_dyn=p["B_dyn"][0], c_dyn=p["c_dyn"][0], dyn_ts=0, dyn_ss=0)
    assert n_tv > cadmm.cadmm_workspace_size(q)[0]


@pytest.mark.parametrize("mutate", [
    lambda p: p.__setitem__("dyn_ts", -1),                                          # negative stride
    lambda p: p.__setitem__("model", 7),                                            # unknown model
    lambda p: p.__setitem__("model", 2),                                            # quadrotor needs 3D, 12/4
    lambda p: p.update(model=1, model_par=np.array([0.0, 2.7])),                    # dt must be > 0
])
def test_invalid_dynamics_rejected(mutate):
    p = workloads.make("c2tv")
    p = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    mutate(p)
    assert _size_code(p) == 1


def test_short_model_arrays_refused_by_the_binding():
    """The C ABI takes raw host pointers, so the binding checks that the
    model arrays hold as many models as the strides address."""
    import paper_2406_07048_amd as cadmm
    p = workloads.make("c2tv")
    p["A_dyn"] = p["A_dyn"][:10]
    with pytest.raises(ValueError):
        cadmm.cadmm_workspace_size(p)


def test_bounds_accepted_and_sized():
    """Bounds add the stage sums and the active-bound slots to the workspace."""
    import paper_2406_07048_amd as cadmm
    p = workloads.make("c2b")
    q = {k: v for k, v in p.items() if k not in ("s_min", "s_max", "u_min", "u_max")}
    assert cadmm.cadmm_workspace_size(p)[0] > cadmm.cadmm_workspace_size(q)[0]
    # infinite entries only: no bounds, no extra memory
    inf = np.inf
    r = dict(q, s_min=np.full(4, -inf), s_max=np.full(4, inf))
    assert cadmm.cadmm_workspace_size(r)[0] == cadmm.cadmm_workspace_size(q)[0]


@pytest.mark.parametrize("mutate", [
    lambda p: p["u_min"].__setitem__(0, 5.0),                                      # min > max
    lambda p: p["s_max"].__setitem__(3, np.nan),                                   # NaN
    lambda p: p["s_min"].__setitem__(0, np.inf),                                   # +inf lower bound
])
def test_invalid_bounds_rejected(mutate):
    p = workloads.make("c2b")
    p = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    mutate(p)
    assert _size_code(p) == 1


def test_bounds_need_the_supported_sizes():
    """The bounded solver's kernels cover n_s <= 12, n_u <= 4."""
    p = workloads.make("c1")
    p = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    n_s = 14
    p.update(n_s=n_s, A_dyn=np.eye(n_s), B_dyn=np.zeros((n_s, 2)), c_dyn=np.zeros(n_s), Q_s=np.eye(n_s),
             x_ref=np.zeros((len(p["obs_ptr"]) - 1, p["N"] + 1, n_s)), x0=np.zeros((len(p["obs_ptr"]) - 1, n_s)))
    assert _size_code(p) == 0
    p["u_max"] = np.array([1.0, 1.0])
    assert _size_code(p) == 1


@pytest.mark.parametrize("name", ["c2sqp", "c3sqp"])
def test_host_model_step_matches_the_oracle(name):
    """cadmm_model_step (the library's FP64 plant step, host code) against the
    oracle's complex-arithmetic model at random states and inputs."""
    import paper_2406_07048_amd as cadmm
    p = workloads.make(name)
    P = oracle.Problem(p)
    rng = np.random.default_rng(3)
    for _ in range(5):
        s = rng.standard_normal(p["n_s"]) * 0.5
        u = rng.standard_normal(p["n_u"]) * 0.5
        F, _, _ = P.model_step(s, u)
        G = cadmm.model_step(p["model"], p["model_par"], s, u)
        assert np.abs(F - G).max() <= 1e-13 * (1 + np.abs(F).max())
    with pytest.raises(cadmm.CadmmError):
        cadmm.model_step(0, p["model_par"], s, u)
