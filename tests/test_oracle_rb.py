"""Pins for the oracle's Rao-Blackwell weights (Thm 3 (2), (5)): the expected
multiplicity of each record given its state, subset and budget.  Checked
against Monte Carlo means of the geometric law (numpy's sampler), against
escape probabilities rebuilt by brute force from the states (numpy energies
of all 2^N states, not the oracle's enumerator), against the target by
enumeration (the ratio estimator of Thm 3 (5)), and against a planted
mistake: ignoring the budget of Alg 6 biases the estimate.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2210_10513_amd import inputs


def _energies(Q):
    """x^T Q x for all 2^N states, state index sum_j x_j 2^j (numpy)."""
    N = Q.shape[0]
    X = ((np.arange(1 << N)[:, None] >> np.arange(N)) & 1).astype(np.float64)
    return np.einsum("si,ij,sj->s", X, Q.astype(np.float64), X)


def _states(x0, actions):
    x = np.array(x0, dtype=np.int64)
    idx = np.empty(len(actions), dtype=np.int64)
    for k, a in enumerate(actions):
        idx[k] = int((x << np.arange(len(x))).sum())
        if a >= 0:
            x[a] ^= 1
    return idx


@pytest.mark.parametrize("p,L", [(0.3, 3), (0.05, 10), (0.9, 2), (0.5, 1), (0.02, -1), (0.4, -1), (0.2, 40)])
def test_expected_multiplicity_is_the_mean_of_the_cut_geometric(p, L):
    """Mean of min(M, L), M = number of trials up to the first success
    (numpy's geometric, support 1, 2, ...), over 4e6 draws."""
    rng = np.random.default_rng(7)
    M = rng.geometric(p, size=4_000_000).astype(np.float64)
    if L >= 0:
        M = np.minimum(M, L)
    se = M.std() / np.sqrt(M.size)
    assert abs(oracle.expected_multiplicity(p, L) - M.mean()) < 5 * se + 1e-12


def test_expected_multiplicity_special_cases_and_closed_form():
    em = oracle.expected_multiplicity
    assert em(1.0, 5) == 1.0 and em(1.0) == 1.0
    assert em(0.37, 1) == 1.0          # one original sample left: M is cut to 1
    assert em(0.37, 0) == 0.0          # no budget left: the record stays with M = 0
    assert em(0.0, 12) == 12.0 and em(0.0) == np.inf
    for p in (0.9, 0.3, 1e-3):
        assert em(p) == pytest.approx(1 / p, rel=1e-15)
        # finite geometric series: sum_{m=1}^{L} (1-p)^(m-1) = (1 - (1-p)^L) / p
        for L in (2, 7, 100, 5000):
            assert em(p, L) == pytest.approx(-np.expm1(L * np.log1p(-p)) / p, rel=1e-12)
        # a long budget reaches the unbudgeted mean
        assert em(p, 10 ** 7) == pytest.approx(1 / p, rel=1e-12)


@pytest.mark.parametrize("dtype", [np.int64, np.float64])
def test_rejection_free_weights_are_one_over_alpha(dtype):
    """RF records: w_k = 1 / alpha(J_k), alpha(x) = (1/N) sum_j
    min(1, pi(x^j)/pi(x)) from brute-force energies."""
    N, beta = 7, 0.35
    Q = inputs.symmetric_int(N, -9, 9, np.int64, seed=4).astype(dtype)
    if dtype == np.float64:
        Q = Q + 0.25 * inputs.symmetric_gauss(N, seed=4).astype(np.float64)
    E = _energies(Q)
    S = np.arange(1 << N)
    alpha = np.mean([np.minimum(1.0, np.exp(-beta * (E[S ^ (1 << j)] - E))) for j in range(N)], axis=0)
    r = oracle.run(Q, beta, oracle.MODE_RF, 300, seed=3, num_chains=3, init="random")
    for c in range(3):
        idx = _states(oracle.random_state(3, c, N), r.action[c])
        assert np.allclose(r.w[c], 1.0 / alpha[idx], rtol=1e-12, atol=0)


@pytest.mark.parametrize("mode", [oracle.MODE_UNBIASED_SYS, oracle.MODE_UNBIASED_RAND])
def test_unbiased_weights_follow_subset_and_budget(mode):
    """Unbiased PNS records: the subset escape probability alpha_i(J_k)
    (Prop 1's per-subset chain) and the budget L rebuilt from the
    multiplicities (L0 at the start and after each stay, minus M after each
    jump) give w_k = (1 - (1 - alpha_i)^L) / alpha_i."""
    N, n, L0, beta, seed = 8, 3, 5, 0.4, 11
    Q = inputs.symmetric_int(N, -7, 7, np.int64, seed=8)
    E = _energies(Q)
    r = oracle.run(Q, beta, mode, 400, n=n, L0=L0, seed=seed, num_chains=2, init="random")
    I = oracle.sys_count(N, n)
    for c in range(2):
        idx = _states(oracle.random_state(seed, c, N), r.action[c])
        L, sub = L0, 0
        members = oracle.sys_subset(N, n, 0) if mode == oracle.MODE_UNBIASED_SYS else \
            oracle.random_subset(seed, c, 0, N, n)
        for k in range(400):
            x = idx[k]
            mem = np.nonzero(members)[0]
            a = np.mean(np.minimum(1.0, np.exp(-beta * (E[x ^ (1 << mem)] - E[x]))))
            assert r.p[c, k] == pytest.approx(a, rel=1e-12)
            want = (1.0 - (1.0 - a) ** L) / a if a < 1 else min(L, 1)
            assert r.w[c, k] == pytest.approx(want, rel=1e-10, abs=1e-300)
            if r.action[c, k] == oracle.STAY:
                L, sub = L0, sub + 1
                members = oracle.sys_subset(N, n, sub % I) if mode == oracle.MODE_UNBIASED_SYS else \
                    oracle.random_subset(seed, c, k + 1, N, n)
            else:
                L -= int(r.M[c, k])


def test_optimization_and_exact_time_weights():
    N = 6
    Q = inputs.symmetric_int(N, -9, 9, np.int64, seed=2)
    r = oracle.run(Q, 0.3, oracle.MODE_OPT, 50, n=N, seed=1, num_chains=2, temperature=0.5)
    assert (r.w == 1.0).all()
    # exact original time T: the last record is cut at the time left
    T = 37
    r = oracle.run(Q, 0.3, oracle.MODE_RF, 200, seed=1, num_chains=3, init="random", orig_time=T)
    for c in range(3):
        k = int(r.n_records[c])
        left = T - np.concatenate([[0], np.cumsum(r.M[c, :k])])[:k]
        want = [oracle.expected_multiplicity(p, L) for p, L in zip(r.p[c, :k], left)]
        assert np.allclose(r.w[c, :k], want, rtol=1e-14)
        assert r.M[c, :k].sum() == T


def _rb_and_m_estimates(Q, beta, mode, K, C, *, n=0, L0=100, seed=0, lib_handle=None):
    r = oracle.run(Q, beta, mode, K, n=n, L0=L0, seed=seed, num_chains=C, init="random", log=False, hist=True,
                   hist_from=K // 10, lib_handle=lib_handle)
    hw = r.hist_w.astype(np.float64)
    return r.hist_rb / r.hist_rb.sum(), hw / hw.sum()


def test_ratio_estimator_with_expected_multiplicities_reaches_pi():
    """Thm 3 (5): sum_k h(J_k) / alpha(J_k) / sum_k 1 / alpha(J_k) -> pi(h).
    RF on N = 6: the weight histogram is within sampling noise of pi, and
    closer than the multiplicity-weighted one of the same records (the
    geometric noise of M is gone)."""
    Q = inputs.symmetric_int(6, -8, 8, np.int64, seed=33)
    pi = exact.target(Q, 0.25)
    rb, mw = _rb_and_m_estimates(Q, 0.25, oracle.MODE_RF, 400, 3000, seed=5)
    assert exact.tv(rb, pi) < 0.01
    assert exact.tv(rb, pi) < exact.tv(mw, pi)


def test_unbiased_estimate_needs_the_budget_cut_weights():
    """Unbiased PNS with a short budget (L0 = 3) at a low temperature: the
    cut means (1 - (1 - p)^L) / p give pi; the uncut 1 / p -- a planted
    mistake in a copy of the oracle -- over-weights the low-alpha states,
    which are left by budget stays, not by jumps."""
    Q = inputs.symmetric_int(6, -8, 8, np.int64, seed=33)
    beta = 0.3
    pi = exact.target(Q, beta)
    rb, mw = _rb_and_m_estimates(Q, beta, oracle.MODE_UNBIASED_SYS, 600, 1500, n=3, L0=3, seed=9)
    assert exact.tv(mw, pi) < 0.01
    assert exact.tv(rb, pi) < 0.01
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        bad = oracle.load_mutant([("orc_expected_multiplicity(p, (unbiased || timed) ? L : -1)",
                                   "orc_expected_multiplicity(p, -1)")], d)
        rb_bad, _ = _rb_and_m_estimates(Q, beta, oracle.MODE_UNBIASED_SYS, 600, 1500, n=3, L0=3, seed=9,
                                        lib_handle=bad)
    assert exact.tv(rb_bad, pi) > 0.06
