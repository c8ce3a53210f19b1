"""GPU parity of the optimization burn-in (Alg 9 / Alg 10, Sec 8): jumps,
energies and the best state X_max against the oracle's MODE_OPT, sampling
after a burn-in against the oracle restarted from the burned-in states, and
the hybrid burn-in of Sec 8.2 converging to the target."""
import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2210_10513_amd import inputs

from parity_util import compare_final, replay_check

pytestmark = pytest.mark.gpu


def _opt_oracle(Q, beta, K, n, T, chains, seed, x0=None, init="zero", layout=oracle.LAYOUT_SYMMETRIC, step0=0):
    Qo = Q.astype(np.int64) if np.issubdtype(Q.dtype, np.integer) else Q.astype(np.float64)
    return oracle.run(Qo, beta, oracle.MODE_OPT, K, n=n, seed=seed, num_chains=chains, x0=x0, init=init,
                      temperature=T, layout=layout, step0=step0)


@pytest.mark.parametrize("mode,n,N,dtype,T", [("rf", 0, 37, np.int32, 0.5), ("rf", 0, 300, np.int16, 2.0),
                                              ("basic", 6, 37, np.int32, 1.0), ("unbiased_sys", 40, 700, np.int16, 0.3),
                                              ("rf", 0, 200, np.float32, 0.8)])
def test_optimization_matches_oracle(mode, n, N, dtype, T):
    from paper_2210_10513_amd.binding import Sampler
    if dtype == np.float32:
        Q = inputs.symmetric_gauss(N, seed=N)
        beta, is_int = 3.0, False
    else:
        Q = inputs.symmetric_int(N, -40, 40, dtype, seed=N)
        beta, is_int = 0.05, True
    C, K = 4, 300
    s = Sampler(Q, beta, n, mode, num_chains=C, seed=17, init="random", log_capacity=K)
    s.optimize(K, T)
    g = {"log": s.read_log(), "cur": s.read_current()}
    xb, eb = s.read_best()
    s.close()
    nn = N if mode == "rf" else n
    rows = list(range(C))
    o, cov = replay_check(g["log"], Q, beta, "opt", rows=rows, is_int=is_int, gcur=g["cur"], n=nn, seed=17,
                          init="random", temperature=T)
    assert cov.compared == C * K and cov.finals == C
    assert (g["log"]["M"] == 1).all()
    assert np.array_equal(xb, o.x_best)
    if is_int:
        assert np.array_equal(eb, o.E_best.astype(np.float64))
    else:
        assert np.allclose(eb, o.E_best, rtol=1e-9, atol=1e-9)


def test_cooling_schedule_and_sampling_after_burn_in():
    """A schedule of two temperatures, then Rejection-Free sampling from the
    burned-in states: the oracle reproduces every step when restarted from
    the same states at the same step counter."""
    from paper_2210_10513_amd.binding import Sampler
    N, C = 120, 3
    Q = inputs.symmetric_int(N, -30, 30, np.int32, seed=5)
    s = Sampler(Q, 0.1, 0, "rf", num_chains=C, seed=3, log_capacity=100)
    s.optimize(100, 2.0).optimize(100, 0.5)
    x_burn = s.read_current()["x"].copy()
    xb, eb = s.read_best()
    s.run(100)
    g = {"log": s.read_log(), "cur": s.read_current()}
    s.close()
    o1 = _opt_oracle(Q, 0.1, 100, N, 2.0, C, 3)
    o2 = _opt_oracle(Q, 0.1, 100, N, 0.5, C, 3, x0=o1.x, step0=100)
    # X_max over both temperatures: the better of the two runs' best states
    best = np.minimum(o1.E_best, o2.E_best)
    assert np.array_equal(eb, best.astype(np.float64))
    assert np.array_equal(x_burn, o2.x)
    rows = list(range(C))
    _, cov = replay_check(g["log"], Q, 0.1, "rf", rows=rows, is_int=True, gcur=g["cur"], seed=3, x0=x_burn,
                          step0=200)
    assert cov.compared == C * 100 and cov.finals == C


def test_adopt_best_moves_chains_to_x_max():
    from paper_2210_10513_amd.binding import Sampler
    N, C = 64, 5
    Q = inputs.symmetric_int(N, -30, 30, np.int32, seed=6)
    s = Sampler(Q, 0.2, 8, "unbiased_sys", num_chains=C, seed=1, init="random", L0=30)
    s.run(50)
    s.optimize(200, 0.3)
    xb, eb = s.read_best()
    s.adopt_best()
    cur = s.read_current()
    assert np.array_equal(cur["x"], xb)
    assert np.array_equal(cur["E"], eb)
    assert (cur["L"] == 30).all()
    Qi = Q.astype(np.int64)
    for c in range(C):
        assert cur["E"][c] == float(xb[c].astype(np.int64) @ Qi @ xb[c].astype(np.int64))
    s.run(20)  # sampling continues from X_max
    assert (s.stats()["anomalies"] == 0).all()
    s.close()


def test_hybrid_burn_in_converges():
    """Sec 8.2: 16 x 16 upper-triangular Q_ij ~ N(0, 1); Optimization PNS
    (halves, n = 8) for K0 = K1 / 20 steps, then Rejection-Free for K1 jumps.
    The last jump-chain states of 100000 chains approach the jump chain's
    stationary law, proportional to alpha(x) pi(x) with alpha the escape
    probability (Thm 3), down to the total variation of 100000 exact draws
    from that law (enumeration)."""
    from paper_2210_10513_amd.binding import Sampler
    N = 16
    Q = inputs.paper_upper_gauss(N, sigma=1.0, seed=72).astype(np.float32)
    E = oracle.enumerate_energies(Q.astype(np.float64), oracle.LAYOUT_UPPER)
    states = np.arange(1 << N)
    alpha = np.mean([np.minimum(1.0, np.exp(-(E[states ^ (1 << j)] - E))) for j in range(N)], axis=0)
    pi = exact.target(Q.astype(np.float64), 1.0, layout=oracle.LAYOUT_UPPER)
    law = alpha * pi / (alpha * pi).sum()
    C = 100_000
    rng = np.random.default_rng(0)
    floor = exact.tv(np.bincount(rng.choice(1 << N, size=C, p=law), minlength=1 << N) / C, law)
    tvs = []
    for K1 in (20, 200, 1000):
        s = Sampler(Q, 1.0, 8, "basic", num_chains=C, seed=K1, init="random", layout="upper")
        s.optimize(max(1, K1 // 20), 1.0)
        x_opt = s.read_current()["x"].copy()
        s.close()
        r = Sampler(Q, 1.0, 0, "rf", num_chains=C, seed=K1 + 1, x0=x_opt, layout="upper")
        r.run(K1)
        x = r.read_current()["x"]
        r.close()
        idx = (x.astype(np.int64) << np.arange(N)).sum(axis=1)
        tvs.append(exact.tv(np.bincount(idx, minlength=1 << N) / C, law))
    assert tvs[0] > tvs[2]
    assert tvs[2] < floor + 0.02, (tvs, floor)
