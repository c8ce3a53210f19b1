"""Exact laws by enumeration, used to pin the oracle (TEST INFRASTRUCTURE).

* ``target(Q, beta)``: pi_beta(x) proportional to exp(-beta x^T Q x) over all
  2^N states (Sec 4 target, sign convention of the oracle's header).
* ``basic_law_graph`` / ``basic_law_qubo``: the limit of the multiplicity-
  weighted sampling distribution of Basic PNS (Alg 3) with a uniformly random
  n-subset each step.  The jump chain moves by the exact one-step kernel
  T(x, y) = E_S[1{y in S} w_y / sum_S w]; its stationary law mu is solved for
  directly; the expected multiplicity is E[M | x] = E_S[n / sum_S w] since M is
  1 + Geometric(p) with p the subset average; the sampling distribution is
  proportional to mu(x) E[M | x] (Sec 2.1 computes Example 1 this way).
* ``tv``: total variation distance, Sec 2.2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import LAYOUT_SYMMETRIC, enumerate_energies, lib


def logsumexp(a: np.ndarray) -> float:
    m = float(np.max(a))
    return m + float(np.log(np.sum(np.exp(a - m))))


def target(Q: np.ndarray, beta: float, layout: int = LAYOUT_SYMMETRIC) -> np.ndarray:
    E = enumerate_energies(Q, layout).astype(np.float64)
    lw = -beta * E
    return np.exp(lw - logsumexp(lw))


def log_partition(Q: np.ndarray, beta: float, layout: int = LAYOUT_SYMMETRIC) -> float:
    E = enumerate_energies(Q, layout).astype(np.float64)
    return logsumexp(-beta * E)


def tv(p: np.ndarray, q: np.ndarray) -> float:
    return 0.5 * float(np.abs(np.asarray(p, dtype=np.float64) - np.asarray(q, dtype=np.float64)).sum())


def empirical(hist: np.ndarray) -> np.ndarray:
    h = np.asarray(hist, dtype=np.float64)
    return h / h.sum()


def basic_onestep(nbr: np.ndarray, logpi: np.ndarray, n: int):
    """(T, EM) of Basic PNS on a D-regular neighbour graph ``nbr`` [S, D]."""
    nbr = np.ascontiguousarray(nbr, dtype=np.int64)
    logpi = np.ascontiguousarray(logpi, dtype=np.float64)
    S, D = nbr.shape
    T = np.zeros((S, D))
    EM = np.zeros(S)
    rc = lib().orc_basic_onestep(S, D, nbr.ctypes.data, logpi.ctypes.data, n, T.ctypes.data, EM.ctypes.data)
    if rc != 0:
        raise ValueError("bad basic_onestep arguments")
    return T, EM


def stationary(nbr: np.ndarray, T: np.ndarray, tol: float = 1e-14, max_iter: int = 200000) -> np.ndarray:
    """Stationary law of the jump chain with kernel T[s, j] -> nbr[s, j].

    The jump chain on the hypercube is periodic (every move changes the
    parity of |x|), so the iteration runs on the lazy kernel (I + T) / 2,
    which has the same stationary law, until successive iterates differ by
    less than ``tol`` in L1.
    """
    S, D = nbr.shape
    rows = np.repeat(np.arange(S), D)
    PT = sp.csr_matrix((T.ravel(), (nbr.ravel(), rows)), shape=(S, S))  # transpose of P
    mu = np.full(S, 1.0 / S)
    for _ in range(max_iter):
        nxt = 0.5 * (mu + PT @ mu)
        nxt /= nxt.sum()
        if np.abs(nxt - mu).sum() < tol:
            return nxt
        mu = nxt
    raise RuntimeError("stationary law did not converge")


def basic_law_graph(nbr: np.ndarray, logpi: np.ndarray, n: int):
    """Returns (P_basic, mu, EM) for a general regular neighbour graph."""
    T, EM = basic_onestep(nbr, logpi, n)
    mu = stationary(nbr, T)
    P = mu * EM
    return P / P.sum(), mu, EM


def hypercube_neighbours(N: int) -> np.ndarray:
    s = np.arange(1 << N, dtype=np.int64)[:, None]
    return s ^ (np.int64(1) << np.arange(N, dtype=np.int64))[None, :]


def basic_law_qubo(Q: np.ndarray, beta: float, n: int, layout: int = LAYOUT_SYMMETRIC):
    """Returns (P_basic, mu, EM, pi) for the QUBO target and single-bit flips."""
    N = Q.shape[0]
    E = enumerate_energies(Q, layout).astype(np.float64)
    logpi = -beta * E
    P, mu, EM = basic_law_graph(hypercube_neighbours(N), logpi, n)
    pi = np.exp(logpi - logsumexp(logpi))
    return P, mu, EM, pi


def second_moments(Q: np.ndarray, beta: float, layout: int = LAYOUT_SYMMETRIC) -> np.ndarray:
    """E_pi[x x^T] by enumeration (N <= 20)."""
    N = Q.shape[0]
    pi = target(Q, beta, layout)
    X = ((np.arange(1 << N)[:, None] >> np.arange(N)[None, :]) & 1).astype(np.float64)
    return X.T @ (pi[:, None] * X)
