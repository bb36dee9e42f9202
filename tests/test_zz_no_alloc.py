"""pair_qp_batch_noalloc (the dual Newton batch with the library's static
device buffer, for callers that cannot allocate) against pair_qp_batch with a
caller workspace (the same two-launch form) and without one (one launch),
through the C ABI: bitwise equal outputs, on two calls in a row, the second
with a smaller batch (the static buffer keeps the first call's contents).
Also: more pairs than the buffer holds are refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from _util import gather_pairs, scaled_pair_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cadmm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2406_07048_amd as m
    m.lib()
    return m


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def batch(n_pairs, seed):
    rp, K, kap, yh, bh = workloads.pair_batch_c4_shape(n_pairs, seed=seed)
    return [to_dev(rp, torch.int32), to_dev(K), to_dev(kap), to_dev(yh), to_dev(bh)], (rp, K, kap, yh, bh)


@pytest.mark.parametrize("n1,n2", [(20000, 3000)])
def test_noalloc_equals_workspace_form(cadmm, n1, n2):
    for n, seed in ((n1, 1), (n2, 2)):
        print(f"[noalloc] {n} pairs (seed {seed})", flush=True)
        args, host = batch(n, seed)
        ws = torch.empty(cadmm.pair_qp_batch_workspace_size(n) + 256, dtype=torch.uint8, device="cuda")
        one = cadmm.pair_qp_batch(*args, 0.1)
        two = cadmm.pair_qp_batch(*args, 0.1, work=ws)
        na = cadmm.pair_qp_batch(*args, 0.1, noalloc=True)
        torch.cuda.synchronize()
        for a, b, c in zip(one, two, na):
            assert torch.equal(a, b) and torch.equal(a, c)
        st = na[3].cpu().numpy()
        assert (st >= 0).all()
        # and the solution is the oracle's (sampled pairs, the scaled dual bar)
        rp, K, kap, yh, bh = host
        y = na[0].cpu().numpy().astype(np.float64)
        worst = 0.0
        for p in range(0, n, max(1, n // 50)):
            sl = slice(rp[p], rp[p + 1])
            nr = int((kap[sl] > 0).sum())
            Kp = K[sl].astype(np.float64)
            A, b = Kp[:nr, 1:], kap[sl][:nr].astype(np.float64)
            Cp, dp = Kp[nr:-1, 1:], Kp[nr:-1, 0]
            yo, it = oracle.pair_qp(A, b, Cp, dp, bh[p, 0] - 1.0, bh[p, 1:], yh[sl].astype(np.float64), 0.1)
            worst = max(worst, scaled_pair_error(Kp, y[sl], yo))
        print(f"   bitwise equal to both other forms; max sweeps {st.max()}; sampled oracle error {worst:.2e}")
        assert worst <= 1e-5


def test_noalloc_refuses_too_many_pairs(cadmm):
    b = cadmm.CadmmPairBatch()
    b.n_pairs = (1 << 19) + 1
    b.dim = 2
    dummy = torch.zeros(16, device="cuda")
    for name in ("row_ptr", "K", "kappa", "yhat", "bhat", "y", "r", "nu", "status"):
        setattr(b, name, dummy.data_ptr())
    b.eps = 0.1
    assert cadmm.lib().pair_qp_batch_noalloc(ctypes.byref(b), None) == cadmm.CADMM_INVALID
