"""GPU parity of in-place coefficient updates (pns_set_q) and snapshot
clearing: after a new Q is swapped in, every chain continues from its state
exactly as the oracle does when restarted from that state on the new Q at
the same step counter."""
import numpy as np
import pytest

from paper_2210_10513_amd import inputs

from parity_util import oracle_run, replay_check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,n,dtype", [("rf", 0, np.int32), ("basic", 7, np.int16), ("rf", 0, np.float32)])
def test_set_q_continues_like_a_restart_on_the_new_q(mode, n, dtype):
    from paper_2210_10513_amd.binding import Sampler
    N, C, K1, K2 = 150, 6, 160, 160  # K1 = K2: the log ring holds steps K1.. in order
    if dtype == np.float32:
        Q1 = inputs.symmetric_gauss(N, seed=1)
        Q2 = inputs.symmetric_gauss(N, seed=2)
        beta, is_int = 2.0, False
    else:
        Q1 = inputs.symmetric_int(N, -40, 40, dtype, seed=1)
        Q2 = inputs.symmetric_int(N, -40, 40, dtype, seed=2)
        beta, is_int = 0.05, True
    s = Sampler(Q1, beta, n, mode, num_chains=C, seed=9, init="random", log_capacity=K2)
    s.run(K1)
    x_mid = s.read_current()["x"].copy()
    s.set_q(Q2)
    cur = s.read_current()
    s.run(K2)
    g = {"log": s.read_log(), "cur": s.read_current()}
    s.close()
    # the log ring holds the last K2 records: those after the swap
    rows = list(range(C))
    o1 = oracle_run(Q1, beta, mode, K1, n=n, seed=9, chains=rows, init="random")
    assert np.array_equal(o1.x, x_mid)
    # fields and energies right after the swap are those of x_mid under Q2
    E_mid = np.einsum("ci,ij,cj->c", x_mid.astype(np.float64), Q2.astype(np.float64), x_mid.astype(np.float64))
    assert np.allclose(cur["E"], E_mid, rtol=1e-12, atol=1e-9)
    _, cov = replay_check(g["log"], Q2, beta, mode, rows=rows, is_int=is_int, gcur=g["cur"], n=n, seed=9, x0=x_mid,
                          step0=K1)
    assert cov.compared == C * K2 and cov.finals == C


def test_set_q_rejects_bad_matrices_and_keeps_the_old_one():
    from paper_2210_10513_amd import binding
    from paper_2210_10513_amd.binding import Sampler
    N = 40
    Q = inputs.symmetric_int(N, -30, 30, np.int32, seed=3)
    a = Sampler(Q, 0.1, 0, "rf", num_chains=3, seed=1)
    b = Sampler(Q, 0.1, 0, "rf", num_chains=3, seed=1)
    a.run(50)
    b.run(50)
    bad = Q.copy()
    bad[0, 5] += 1
    with pytest.raises(binding.PNSError) as ei:
        a.set_q(bad)
    assert ei.value.code == binding.PNS_EINVAL and "symmetric" in str(ei.value)
    huge = (np.ones((N, N)) * 2e8).astype(np.int32)
    with pytest.raises(binding.PNSError) as ei:
        a.set_q(huge)
    assert ei.value.code in (binding.PNS_EINVAL, binding.PNS_EUNSUPPORTED)
    a.run(50)
    b.run(50)
    assert np.array_equal(a.read_current()["x"], b.read_current()["x"])
    assert np.array_equal(a.read_current()["E"], b.read_current()["E"])
    a.close()
    b.close()


def test_snapshots_clear_forgets_old_snapshots():
    from paper_2210_10513_amd.binding import Sampler
    Q = inputs.symmetric_int(30, -30, 30, np.int32, seed=4)
    s = Sampler(Q, 0.1, 0, "rf", num_chains=4, seed=1, snapshot_every=2, snapshot_capacity=5)
    s.run(10)
    s.snapshots_clear()
    xs, ms, _, cnt = s.read_snapshots()
    assert cnt == 0 and (ms == 0).all()
    G, sm = s.snapshot_moments()
    assert sm == 0.0 and (G == 0).all()
    s.run(4)
    xs, ms, _, cnt = s.read_snapshots()
    assert cnt == 2 and (ms[:, :2] > 0).all() and (ms[:, 2:] == 0).all()
    s.close()
