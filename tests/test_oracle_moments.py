"""Pins of the differentiation oracle (oracle/moments.py) against what the
mathematics fixes: invariants of X^T diag(m) X, closed forms of log Z and
E[x x^T] for independent bits, a brute-force loop over the states, and
finite differences of log Z.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact, moments


def _sym_int(N, seed, lo=-6, hi=6):
    rng = np.random.default_rng(seed)
    U = rng.integers(lo, hi + 1, size=(N, N))
    return np.triu(U) + np.triu(U, 1).T


def test_weighted_moments_invariants():
    rng = np.random.default_rng(1)
    K, N = 60, 7
    X = rng.integers(0, 2, size=(K, N)).astype(np.uint8)
    m = rng.integers(0, 1000, size=K)
    G = moments.weighted_moments(X, m)
    assert G.dtype == np.int64
    assert np.array_equal(G, G.T)
    # the diagonal is the weighted count of ones of each bit (x_i^2 = x_i)
    assert np.array_equal(np.diag(G), (m[:, None] * X).sum(axis=0))
    # 1^T G 1 = sum_k m_k (number of ones in record k)^2
    assert G.sum() == int((m * X.sum(axis=1).astype(np.int64) ** 2).sum())
    # records that are unit vectors give a diagonal matrix of their weights
    E = np.eye(N, dtype=np.uint8)
    assert np.array_equal(moments.weighted_moments(E, np.arange(1, N + 1)), np.diag(np.arange(1, N + 1)))
    # positive semidefinite
    assert np.linalg.eigvalsh(G.astype(float)).min() > -1e-9
    # float weights with integral values give the same matrix
    assert np.array_equal(moments.weighted_moments(X, m.astype(np.float64)), G.astype(np.float64))
    # G_ij counts the weight of records with both bits set
    i, j = 2, 5
    assert G[i, j] == int(m[(X[:, i] == 1) & (X[:, j] == 1)].sum())
    pairs = [(0, 0), (2, 5), (6, 1), (3, 3)]
    assert np.array_equal(moments.weighted_moment_entries(X, m, pairs), [G[a, b] for a, b in pairs])


@pytest.mark.parametrize("N,seed", [(1, 0), (4, 1), (7, 2)])
def test_log_partition_matches_state_loop(N, seed):
    Q = _sym_int(N, seed)
    for beta in (0.0, 0.3, 1.7):
        assert math.isclose(exact.log_partition(Q, beta), moments.log_partition_loop(Q, beta), rel_tol=1e-12,
                            abs_tol=1e-12)
    Qf = np.random.default_rng(seed).standard_normal((N, N))
    Qf = (Qf + Qf.T) / 2
    assert math.isclose(exact.log_partition(Qf, 0.8), moments.log_partition_loop(Qf, 0.8), rel_tol=1e-12)


def test_log_partition_closed_forms():
    N = 9
    assert math.isclose(exact.log_partition(np.zeros((N, N), np.int64), 2.0), N * math.log(2.0), rel_tol=1e-14)
    d = np.array([3, -2, 0, 5, -7, 1, 4, -1, 2])
    beta = 0.45
    want = sum(math.log1p(math.exp(-beta * v)) for v in d)
    assert math.isclose(exact.log_partition(np.diag(d), beta), want, rel_tol=1e-13)


def test_second_moments_of_independent_bits():
    d = np.array([2, -1, 0, 3, -4])
    beta = 0.7
    S = exact.second_moments(np.diag(d), beta)
    p = 1.0 / (1.0 + np.exp(beta * d))
    want = np.outer(p, p)
    np.fill_diagonal(want, p)
    assert np.allclose(S, want, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", [3, 4])
def test_gradient_matches_finite_differences_of_state_loop(seed):
    """d log Z / dQ: a symmetric perturbation of Q_ij and Q_ji (i != j) by
    eps moves log Z by -2 beta E[x_i x_j] eps; of Q_ii by -beta E[x_i] eps."""
    N = 5
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((N, N))
    Q = (Q + Q.T) / 2
    beta = 0.9
    g = moments.grad_log_partition(Q, beta)
    eps = 1e-5
    for i, j in [(0, 0), (1, 3), (2, 4), (4, 4), (0, 1)]:
        Dp = Q.copy()
        Dm = Q.copy()
        Dp[i, j] += eps
        Dm[i, j] -= eps
        if i != j:
            Dp[j, i] += eps
            Dm[j, i] -= eps
        fd = (moments.log_partition_loop(Dp, beta) - moments.log_partition_loop(Dm, beta)) / (2 * eps)
        want = g[i, j] * (2 if i != j else 1)
        assert abs(fd - want) < 1e-7, (i, j, fd, want)


def test_nll_gradient_and_moment_matching():
    """The NLL gradient is beta (E_data - E_model): zero when the data moments
    are the model's own, and equal to finite differences of the loss."""
    N = 4
    Q = _sym_int(N, 7).astype(np.float64) / 3
    beta = 1.1
    Sm = exact.second_moments(Q, beta)
    loss, grad = moments.nll(Q, beta, Sm)
    assert np.abs(grad).max() < 1e-12
    rng = np.random.default_rng(0)
    data = exact.second_moments(_sym_int(N, 8).astype(np.float64) / 3, beta)
    loss, grad = moments.nll(Q, beta, data)
    eps = 1e-6
    D = np.zeros((N, N))
    D[1, 2] = D[2, 1] = eps
    fd = (moments.nll(Q + D, beta, data)[0] - moments.nll(Q - D, beta, data)[0]) / (2 * eps)
    assert abs(fd - 2 * grad[1, 2]) < 1e-7
    # the loss at the data-generating Q is below the loss at a perturbed Q
    Q0 = _sym_int(N, 8).astype(np.float64) / 3
    l0 = moments.nll(Q0, beta, data)[0]
    assert l0 < moments.nll(Q0 + 0.3 * rng.standard_normal((N, N)), beta, data)[0]


def test_jump_chain_weighted_moments_estimate_second_moments():
    """The multiplicity-weighted moments of an oracle Rejection-Free run
    converge to E_pi[x x^T] (the estimator the backward pass uses)."""
    N = 6
    Q = _sym_int(N, 11)
    beta = 0.4
    K = 40000
    r = oracle.run(Q.astype(np.int64), beta, oracle.MODE_RF, K, seed=3, num_chains=1, log=True)
    # the state of each record: replay the flips from x = 0
    x = np.zeros(N, np.uint8)
    X = np.zeros((K, N), np.uint8)
    for k in range(K):
        X[k] = x
        a = r.action[0, k]
        if a >= 0:
            x[a] ^= 1
    G = moments.weighted_moments(X[K // 10:], r.M[0, K // 10:])
    est = G / r.M[0, K // 10:].sum()
    assert np.abs(est - exact.second_moments(Q, beta)).max() < 0.02
