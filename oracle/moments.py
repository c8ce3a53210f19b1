"""Oracle of the differentiation path (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline
may import this module.

The target pi_beta(x) = exp(-beta x^T Q x) / Z(Q, beta) (Sec 4, sign
convention of the oracle) gives, for every entry of a matrix Q whose entries
are free parameters,

    d log Z / d Q_ij = -beta E_pi[x_i x_j],

so grad_Q log Z = -beta E_pi[x x^T].  The jump chain (J_k, M_k) of
Rejection-Free / Unbiased PNS estimates E_pi[f] by sum_k M_k f(J_k) /
sum_k M_k (Sec 1.2, the multiplicity list replaces the repeated states), so
the estimate of E_pi[x x^T] from records (x_k, m_k) is G / sum_k m_k with

    G = sum_k m_k x_k x_k^T = X^T diag(m) X.

Functions
* ``weighted_moments(X, m)``: G, written out from that definition in int64
  (integer m) or float64.
* ``weighted_moment_entries(X, m, pairs)``: chosen entries of G one by one.
* ``log_partition_loop(Q, beta)``: log Z by a plain Python loop over the
  2^N states (small N), independent of the C enumerator.
* ``grad_log_partition(Q, beta)``: -beta E_pi[x x^T] by enumeration.
* ``nll(Q, beta, data_moments)``: average negative log-likelihood of data
  with second moments E_data[x x^T] = data_moments, and its gradient
  beta (E_data[x x^T] - E_pi[x x^T]) -- the maximum-likelihood fit of a
  QUBO/Boltzmann model matches the model's second moments to the data's.
"""
from __future__ import annotations

import math

import numpy as np

from . import LAYOUT_SYMMETRIC
from .exact import log_partition, second_moments


def weighted_moments(X: np.ndarray, m: np.ndarray) -> np.ndarray:
    """G = sum_k m_k x_k x_k^T for records X [K, N] of 0/1 and weights m [K]."""
    X = np.asarray(X)
    m = np.asarray(m)
    if np.issubdtype(m.dtype, np.integer):
        mi = m.astype(np.int64)
        if X.shape[0] == 0 or int(np.abs(mi).max()) * X.shape[0] < 2 ** 53:
            # every partial sum is an integer below 2^53: FP64 is exact
            Xf = X.astype(np.float64)
            return np.rint((Xf * mi.astype(np.float64)[:, None]).T @ Xf).astype(np.int64)
        Xi = X.astype(np.int64)
        return (Xi * mi[:, None]).T @ Xi
    Xf = X.astype(np.float64)
    return (Xf * m.astype(np.float64)[:, None]).T @ Xf


def weighted_moment_entries(X: np.ndarray, m: np.ndarray, pairs) -> np.ndarray:
    """G_ij = sum of m_k over the records with bits i and j both set, for each
    (i, j) in ``pairs`` (entries of a G too large to form)."""
    X = np.asarray(X)
    m = np.asarray(m)
    out = []
    for i, j in pairs:
        both = (X[:, i] != 0) & (X[:, j] != 0)
        out.append(m[both].sum())
    return np.asarray(out)


def log_partition_loop(Q: np.ndarray, beta: float) -> float:
    """log sum_x exp(-beta x^T Q x) by a Python loop over every state."""
    N = Q.shape[0]
    Qf = np.asarray(Q, dtype=np.float64)
    lw = []
    for s in range(1 << N):
        x = np.array([(s >> j) & 1 for j in range(N)], dtype=np.float64)
        lw.append(-beta * float(x @ Qf @ x))
    top = max(lw)
    return top + math.log(sum(math.exp(v - top) for v in lw))


def grad_log_partition(Q: np.ndarray, beta: float, layout: int = LAYOUT_SYMMETRIC) -> np.ndarray:
    """-beta E_pi[x x^T] (N <= 20)."""
    return -beta * second_moments(Q, beta, layout)


def nll(Q: np.ndarray, beta: float, data_moments: np.ndarray):
    """(loss, gradient) of the average negative log-likelihood
    beta <Q, E_data[x x^T]> + log Z(Q), by enumeration (N <= 20)."""
    loss = beta * float(np.sum(Q * data_moments)) + log_partition(Q, beta)
    grad = beta * (data_moments - second_moments(Q, beta))
    return loss, grad
