"""GPU parity of runs of exactly T original samples (pns_run_original) and
of parallel-tempering swap rounds (pns_pt_swap) against the oracle, and the
per-temperature targets under tempering (enumeration)."""
import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2210_10513_amd import inputs

from parity_util import compare_final, replay_check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,n,dtype", [("rf", 0, np.int32), ("basic", 5, np.int16), ("rf", 0, np.float32)])
def test_original_time_run_matches_oracle(mode, n, dtype):
    from paper_2210_10513_amd.binding import Sampler
    N, C, T = 90, 6, 400
    if dtype == np.float32:
        Q = inputs.symmetric_gauss(N, seed=3)
        beta, is_int = 2.0, False
    else:
        Q = inputs.symmetric_int(N, -30, 30, dtype, seed=3)
        beta, is_int = 0.08, True
    s = Sampler(Q, beta, n, mode, num_chains=C, seed=8, init="random", log_capacity=T)
    s.run_original(T)
    log = s.read_log()
    cur = s.read_current()
    s.close()
    Qo = Q.astype(np.int64) if is_int else Q.astype(np.float64)
    o = oracle.run(Qo, beta, oracle.MODE_RF if mode == "rf" else oracle.MODE_BASIC, T, n=n, seed=8, num_chains=C,
                   init="random", orig_time=T)
    assert np.array_equal(cur["step"], o.n_records)
    _, cov = replay_check(log, Q, beta, mode, rows=list(range(C)), is_int=is_int, lengths=cur["step"], gcur=cur,
                          n=n, seed=8, init="random", orig_time=T)
    assert cov.compared == int(o.n_records.sum()) and cov.finals == C
    for c in range(C):
        assert log["M"][c, :int(o.n_records[c])].sum() == T


def test_tempering_sweeps_match_oracle():
    """Sweeps of 7 original samples and swap rounds over groups of 4
    temperatures: betas, ladders, accepted flags, states and energies equal
    the oracle's."""
    from paper_2210_10513_amd.binding import Sampler
    N, T, groups = 40, 4, 30
    C = T * groups
    Q = inputs.symmetric_int(N, -20, 20, np.int32, seed=9)
    ladder_b = inputs.beta_ladder(T, 0.02, 0.5)
    betas = np.tile(ladder_b[::-1], groups).astype(np.float64)  # reverse order: the ladder sorts them
    s = Sampler(Q, betas, 0, "rf", num_chains=C, seed=13, init="random")
    xo = np.stack([oracle.random_state(13, c, N) for c in range(C)])
    bo = betas.copy()
    lad = np.zeros(C, np.int32)
    for g in range(groups):
        lad[g * T:(g + 1) * T] = np.argsort(bo[g * T:(g + 1) * T], kind="stable")
    steps = np.zeros(C, np.int64)
    for sweep in range(12):
        s.run_original(7)
        acc = s.pt_swap(T, sweep)
        r = oracle.run(Q.astype(np.int64), bo, oracle.MODE_RF, 7, seed=13, num_chains=C, x0=xo, step0=steps,
                       orig_time=7, log=False)
        xo = r.x
        steps = steps + r.n_records
        acc_o = oracle.pt_round(r.E_final, bo, lad, T, seed=13, round_=sweep)
        assert np.array_equal(acc, acc_o), sweep
    assert np.array_equal(s.betas(), bo)
    assert np.array_equal(s.ladder(), lad)
    cur = s.read_current()
    assert np.array_equal(cur["x"], xo)
    assert np.array_equal(cur["step"], steps)
    s.close()


def test_tempering_keeps_each_temperature_at_its_target():
    """Two temperatures, 6000 groups, RF sweeps of 4 original samples
    alternated with swaps, started from exact draws: the state held at each
    temperature follows pi at that temperature (enumeration)."""
    from paper_2210_10513_amd.binding import Sampler
    Q = inputs.symmetric_int(6, -8, 8, np.int32, seed=33)
    ladder_b = np.array([0.15, 0.8])
    T, groups = 2, 6000
    C = T * groups
    pis = [exact.target(Q.astype(np.int64), b) for b in ladder_b]
    rng = np.random.default_rng(2)
    x0 = np.zeros((C, 6), np.uint8)
    for t in range(T):
        idx0 = rng.choice(64, size=groups, p=pis[t])
        x0[t::T] = ((idx0[:, None] >> np.arange(6)) & 1).astype(np.uint8)
    s = Sampler(Q, np.tile(ladder_b, groups), 0, "rf", num_chains=C, seed=5, x0=x0)
    swaps = 0
    for sweep in range(25):
        s.run_original(4)
        swaps += int(s.pt_swap(T, sweep).sum())
    x = s.read_current()["x"]
    lad = s.ladder()
    s.close()
    assert swaps > 0.05 * groups * 25 / 2
    for t in range(T):
        chains = np.arange(groups) * T + lad[t::T]
        idx = (x[chains].astype(np.int64) << np.arange(6)).sum(axis=1)
        floor = exact.tv(np.bincount(rng.choice(64, size=groups, p=pis[t]), minlength=64) / groups, pis[t])
        assert exact.tv(np.bincount(idx, minlength=64) / groups, pis[t]) < floor + 0.02
