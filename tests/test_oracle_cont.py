"""Pins for the continuous Unbiased PNS oracle (Alg 7 on the donut target of
Sec 7).  The oracle is checked against: the standard normal law of its
offset draws (Kolmogorov-Smirnov, moments); every step rebuilt by brute force
in numpy from the logged states (target density, escape probability over the
2P neighbours x +- delta_j of the current set, the budget of Alg 7, the
expected multiplicities); the exact moments of the donut law (quadrature)
estimated over an exact original-time window from exact draws, where the
original chain stays stationary (Prop 1: each set's kernel keeps pi); and two
planted mistakes (uncapped acceptance weights, one-sided neighbour sets) that
those estimates catch.  CPU only."""
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import donut
from paper_2210_10513_amd import inputs


def _logpi(x, mu0, sigma):
    u = (np.asarray(x) ** 2).sum(-1)
    return -(u - mu0) ** 2 / (2 * sigma ** 2)


def test_offsets_are_independent_standard_normals():
    d, P = 3, 25
    D = np.concatenate([oracle.cont_offsets(17, c, s, P, d) for c in range(20) for s in range(20)])
    v = D.reshape(-1)
    assert stats.kstest(v, "norm").pvalue > 1e-4
    n = v.size
    assert abs(v.mean()) < 5 / np.sqrt(n)
    assert abs(v.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(v, fisher=False) - 3) < 5 * np.sqrt(24 / n)
    c = np.corrcoef(D.T)
    assert np.abs(c - np.eye(d)).max() < 5 / np.sqrt(D.shape[0])
    # sets and chains draw different offsets
    assert not np.allclose(oracle.cont_offsets(17, 0, 0, P, d), oracle.cont_offsets(17, 0, 1, P, d))
    assert not np.allclose(oracle.cont_offsets(17, 0, 0, P, d), oracle.cont_offsets(17, 1, 0, P, d))


@pytest.mark.parametrize("d,sigma,P,L0", [(2, 0.3, 5, 60), (3, 1.0, 4, 25), (1, 0.5, 2, 10)])
def test_every_step_follows_alg7_by_brute_force(d, sigma, P, L0):
    mu0, seed, C, K = 9.0, 23, 3, 400
    x0 = inputs.donut_draws(C, d, mu0, sigma, seed=3)
    r = oracle.cont_run(x0, K, mu0=mu0, sigma=sigma, pairs=P, L0=L0, seed=seed, log_states=True)
    for c in range(C):
        L, s = L0, 0
        D = oracle.cont_offsets(seed, c, s, P, d)
        block_M = 0
        x = x0[c].copy()
        for k in range(K):
            assert np.array_equal(r.xs[c, k], x)
            lp = _logpi(x, mu0, sigma)
            assert r.E[c, k] == pytest.approx(lp, rel=1e-12, abs=1e-12)
            nb = np.concatenate([x + D, x - D])        # x + delta_j, then x - delta_j
            w = np.minimum(1.0, np.exp(_logpi(nb, mu0, sigma) - lp))
            p = w.mean()
            assert r.p[c, k] == pytest.approx(p, rel=1e-12)
            em = -np.expm1(L * np.log1p(-p)) / p if 0 < p < 1 else (1.0 if p >= 1 else float(L))
            assert r.w[c, k] == pytest.approx(em, rel=1e-10)
            q = r.q[c, k]
            M = int(r.M[c, k])
            block_M += M
            if r.action[c, k] == oracle.STAY:
                assert q >= L and M == L
                assert block_M == L0                 # a set is used for exactly L0 original samples
                block_M, L, s = 0, L0, s + 1
                D = oracle.cont_offsets(seed, c, s, P, d)
            else:
                j = int(r.action[c, k])
                assert q < L and M == int(np.floor(q)) + 1
                # the choice is the first neighbour whose running weight sum exceeds U2 * S
                U2 = oracle.uniforms(seed, c, k)[1]
                cs = np.cumsum(w)
                assert cs[j] > U2 * cs[-1] and (j == 0 or cs[j - 1] <= U2 * cs[-1] * (1 + 1e-12))
                L -= M
                x = x + D[j] if j < P else x - D[j - P]
        assert np.allclose(r.x[c], x, rtol=0, atol=0)
        assert r.L[c] == L and r.set[c] == s


def _window_estimates(r, T, mu0):
    """(1/T) sum_{t < T} h(X_t) per chain, from the records (J_k, M_k): the
    original chain sits at J_k for M_k consecutive samples."""
    C, K, d = r.xs.shape
    start = np.concatenate([np.zeros((C, 1), np.int64), np.cumsum(r.M, axis=1)[:, :-1]], axis=1)
    wt = np.minimum(np.clip(T - start, 0, None), r.M).astype(np.float64)
    assert (wt.sum(1) == T).all(), "run too short for the window"
    x = r.xs
    u = (x ** 2).sum(-1, keepdims=True)
    hs = {"x": x, "x2": x ** 2, "x4": x ** 4, "pos": (x > 0).astype(np.float64), "u": u, "v": (u - mu0) ** 2}
    return {k: (wt[:, :, None] * h).sum(1) / T for k, h in hs.items()}


def _z_scores(est, exact):
    z = {}
    for k, v in est.items():
        se = v.std(0, ddof=1) / np.sqrt(v.shape[0])
        z[k] = np.abs(v.mean(0) - exact[k]) / se
    return z


def _exact(d, mu0, sigma):
    ex = donut.coordinate_moments(d, mu0, sigma)
    Eu, Eu2 = donut.radial_moments(d, mu0, sigma)
    ex["u"] = Eu
    ex["v"] = Eu2 - 2 * mu0 * Eu + mu0 ** 2
    return ex


def _run_window(d, mu0, sigma, P, L0, C, T, K, seed, lib_handle=None):
    x0 = inputs.donut_draws(C, d, mu0, sigma, seed=seed)
    r = oracle.cont_run(x0, K, mu0=mu0, sigma=sigma, pairs=P, L0=L0, seed=seed + 1, log_states=True,
                        lib_handle=lib_handle)
    return _window_estimates(r, T, mu0), r


@pytest.mark.parametrize("d,sigma,P,L0,T,K", [(2, 0.1, 25, 1000, 20000, 3000), (3, 1.0, 25, 200, 4000, 3000)])
def test_exact_time_estimates_match_the_donut_moments(d, sigma, P, L0, T, K):
    """From exact draws of pi the original chain stays at pi (each set's
    kernel keeps it), so (1/T) sum_t h(X_t) is unbiased: 400 independent
    chains give z-scores below 5 for x, x^2, x^4, 1(x > 0), |x|^2 and
    (|x|^2 - mu0)^2 (Sec 7's workload: d = 2, mu0 = 9, sigma = 0.1,
    |N| = 50, L0 = 1000; and a wide donut in d = 3)."""
    est, _ = _run_window(d, 9.0, sigma, P, L0, 400, T, K, seed=5)
    z = _z_scores(est, _exact(d, 9.0, sigma))
    for k, v in z.items():
        assert (v < 5).all(), (k, v)


def test_expected_multiplicity_sums_estimate_the_radius():
    """The estimator sums kept per chain (weights M and the expected
    multiplicities, Thm 3 (5)) estimate E[|x|^2] within 5 standard errors of
    the per-chain ratio estimates."""
    d, mu0, sigma = 2, 9.0, 0.1
    x0 = inputs.donut_draws(400, d, mu0, sigma, seed=6)
    r = oracle.cont_run(x0, 3000, mu0=mu0, sigma=sigma, pairs=25, L0=1000, seed=9, log=False)
    Eu = donut.radial_moments(d, mu0, sigma)[0]
    for row in (0, 1):
        S = r.sums[:, row]
        u = S[:, 1 + d:1 + 2 * d].sum(1) / S[:, 0]
        assert abs(u.mean() - Eu) < 5 * u.std(ddof=1) / np.sqrt(u.size)
    # both weightings cover about the same number of original samples
    assert np.all(r.sums[:, 0, 0] > 0)
    assert abs(r.sums[:, 1, 0].sum() / r.sums[:, 0, 0].sum() - 1) < 0.01


@pytest.mark.parametrize("name,replacements", [
    ("uncapped acceptance weights", [("w[j] = l < 0.0 ? exp(l) : 1.0;", "w[j] = exp(l);")]),
    ("one-sided neighbour sets", [("const double sgn = j < P ? 1.0 : -1.0;", "const double sgn = 1.0;"),
                                  ("const double sgn = c < P ? 1.0 : -1.0;", "const double sgn = 1.0;")]),
])
def test_planted_mistakes_are_caught(name, replacements):
    with tempfile.TemporaryDirectory() as dd:
        bad = oracle.load_mutant(replacements, dd)
        est, _ = _run_window(2, 9.0, 0.1, 25, 1000, 400, 20000, 3000, seed=5, lib_handle=bad)
    z = _z_scores(est, _exact(2, 9.0, 0.1))
    assert z["v"].max() > 10, (name, z["v"])
