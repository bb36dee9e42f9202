"""The paper's own route for the dual-update QP on the GPU (Sec. IV-C: the
equality eliminated, eq. const_least_square_ineq; the KKT conditions as the
LCP of eq. linear_complementarity_problem; Lemke's method), offered by the
stateless batch entry point as the alternative to the dual Newton solver.

Checked through the C ABI against the FP64 oracle's active-set solution of
the same proximal QP (unique) on pairs of oracle iterates of the 2D and 3D
workloads, against the GPU's dual Newton on the same batch, and at the edges
(the largest pair, a pair already at its optimum, sizes outside the tableau).
Bar: the scaled dual bar of the other parity tests, 1e-5 per pair."""
import numpy as np
import pytest

import oracle
import workloads
from _util import K_rows, gather_pairs, scaled_pair_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_DUAL = 1e-5


@pytest.fixture(scope="module")
def cadmm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2406_07048_amd as m
    m.lib()
    return m


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run(cadmm, row_ptr, K, kap, yh, bh, eps, solver):
    y, r, nu, st = cadmm.pair_qp_batch(to_dev(row_ptr, torch.int32), to_dev(K), to_dev(kap), to_dev(yh),
                                       to_dev(bh), eps, solver=solver)
    torch.cuda.synchronize()
    return (y.cpu().numpy().astype(np.float64), r.cpu().numpy().astype(np.float64), nu.cpu().numpy(),
            st.cpu().numpy())


@pytest.mark.parametrize("name,k", [("c1", 0), ("c1", 5), ("c2", 3), ("c2", 60), ("c3", 3), ("c3", 30)])
def test_lemke_batch_parity(cadmm, name, k):
    prob = workloads.make(name)
    print(f"[lemke batch] {name} iterate {k}", flush=True)
    P = oracle.Problem(prob)
    st = P.init_state()
    if k:
        P.run(st, k)
    layout = workloads.block_layout(prob)
    nb = len(layout[0])
    rng = np.random.default_rng(0)
    pairs = [(int(rng.integers(nb)), int(rng.integers(1, prob["N"] + 1))) for _ in range(400)]
    row_ptr, K, kap, yh, bh, geo = gather_pairs(prob, st, pairs, layout)
    eps = prob["eps_prox"]
    yl, rl, nul, stl = run(cadmm, row_ptr, K, kap, yh, bh, eps, cadmm.CADMM_PAIR_LEMKE)
    yn, rn, nun, stn = run(cadmm, row_ptr, K, kap, yh, bh, eps, cadmm.CADMM_PAIR_NEWTON)
    worst = worst_ab = 0.0
    for p, (A, bb, Cp, dp, z, xi) in enumerate(geo):
        sl = slice(row_ptr[p], row_ptr[p + 1])
        yo, it = oracle.pair_qp(A, bb, Cp, dp, z, xi, yh[sl], eps)
        Kp = K[sl]
        worst = max(worst, scaled_pair_error(Kp, yl[sl], yo))
        worst_ab = max(worst_ab, scaled_pair_error(Kp, yl[sl], yn[sl]))
        ro = Kp.T @ yo + bh[p]
        assert np.abs(rl[p] - ro).max() <= 1e-5 * (1.0 + (np.abs(Kp).sum(1) * yo).sum())
    print(f"   Lemke vs oracle: worst scaled dual error {worst:.2e}; vs the dual Newton {worst_ab:.2e}; "
          f"pivots mean {stl[stl >= 0].mean():.1f} max {stl.max()}", flush=True)
    assert (stl >= 0).all()
    assert worst <= TOL_DUAL


def test_lemke_batch_edges(cadmm):
    """The largest pair (8 + 32 + 1 rows), a pair at its optimum (the scale-LP
    certificate of a disjoint pair with zero multipliers: y = yhat), and a
    pair of 42 rows, outside the tableau (status -3, other pairs unaffected)."""
    rng = np.random.default_rng(4)
    A = np.concatenate([np.eye(2), -np.eye(2), [[0.6, 0.8], [-0.6, 0.8], [0.6, -0.8], [-0.6, -0.8]]])
    b = np.r_[1.0, 1.0, 1.0, 1.0, 1.3, 1.3, 1.3, 1.3]
    ang = np.sort(rng.uniform(0, 2 * np.pi, 32))
    Cp = np.stack([np.cos(ang), np.sin(ang)], 1)
    dp = 1.0 + Cp @ np.array([4.0, 1.0])
    K1 = K_rows(A, Cp, dp)
    yh1 = np.abs(rng.normal(size=len(K1)))
    bh1 = np.array([1.3, 0.2, -0.1])
    Cb = np.concatenate([np.eye(2), -np.eye(2)])
    db = np.r_[5.0, 1.0, -4.0, 1.0]
    alpha, _, lam, mu, gap, _ = oracle.scale_lp(A, b, Cb, db)
    K2 = K_rows(A, Cb, db)
    yh2 = np.r_[lam, mu, alpha - 1.0]
    bh2 = np.array([1.0, 0.0, 0.0])
    K3 = np.concatenate([K1, [[0.5, 0.1, 0.2]]])           # 42 rows
    yh3 = np.r_[yh1, 0.1]
    kap1 = np.r_[b, np.zeros(len(dp) + 1)]
    kap2 = np.r_[b, np.zeros(len(db) + 1)]
    kap3 = np.r_[kap1, 0.0]
    row_ptr = np.cumsum([0, len(K1), len(K2), len(K3)]).astype(np.int32)
    y, r, nu, st = run(cadmm, row_ptr, np.concatenate([K1, K2, K3]), np.r_[kap1, kap2, kap3],
                       np.r_[yh1, yh2, yh3], np.stack([bh1, bh2, bh1]), 0.1, cadmm.CADMM_PAIR_LEMKE)
    yo1, _ = oracle.pair_qp(A, b, Cp, dp, bh1[0] - 1.0, bh1[1:], yh1, 0.1)
    e1 = scaled_pair_error(K1, y[:len(K1)], yo1)
    e2 = scaled_pair_error(K2, y[row_ptr[1]:row_ptr[2]], yh2)
    print(f"   largest pair {e1:.2e} ({st[0]} pivots); optimal centre {e2:.2e} ({st[1]} pivots); 42 rows: {st[2]}")
    assert st[0] >= 0 and e1 <= TOL_DUAL
    assert st[1] >= 0 and e2 <= TOL_DUAL
    assert st[2] == -3
