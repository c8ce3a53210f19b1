"""Seeded synthetic QUBO inputs shared by the tests, the benchmark and the
oracle runs.  This module draws only the problem data (matrices, inverse
temperatures, initial states); it holds none of the sampler's arithmetic.

The paper's experiments use synthetic random QUBO matrices (Sec 4: 16x16
upper-triangular Q_ij ~ N(0, 10^2); Sec 8.2: N(0, 1)) and the 16-state
example of Sec 2.2; the workloads below keep those generators and scale them
to the sizes the sampler is benchmarked at.  Target convention throughout:
pi_beta(x) proportional to exp(-beta x^T Q x).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

SEED_BASE = 2210105130


def _rng(tag: int, seed: int | None) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + tag if seed is None else seed)


def _mirror_upper(Q: np.ndarray, block: int = 256) -> np.ndarray:
    """Copy the strict upper triangle of Q onto the lower one, in place, in
    square blocks (a whole-matrix transpose is slow at N = 16384)."""
    N = Q.shape[0]
    for i0 in range(0, N, block):
        i1 = min(N, i0 + block)
        d = Q[i0:i1, i0:i1]
        d += np.triu(d, 1).T
        for j0 in range(i1, N, block):
            j1 = min(N, j0 + block)
            Q[j0:j1, i0:i1] = Q[i0:i1, j0:j1].T
    return Q


def symmetric_int(N: int, lo: int, hi: int, dtype=np.int32, seed: int | None = None, density: float = 1.0,
                  tag: int = 0) -> np.ndarray:
    """Dense symmetric integer QUBO: entries i <= j iid uniform on {lo..hi}
    (optionally kept with probability ``density``), mirrored below."""
    rng = _rng(tag, seed)
    draw = np.int16 if -32768 <= lo and hi <= 32766 else np.int64
    U = rng.integers(lo, hi + 1, size=(N, N), dtype=draw)
    if density < 1.0:
        U *= rng.random((N, N), dtype=np.float32) < np.float32(density)
    Q = _mirror_upper(np.triu(U))
    return Q.astype(dtype, copy=False)


def symmetric_gauss(N: int, seed: int | None = None, tag: int = 0, dtype=np.float32) -> np.ndarray:
    """Q = (A + A^T) / 2 with A_ij iid N(0, 1) / sqrt(N), in float32."""
    rng = _rng(tag, seed)
    A = rng.standard_normal((N, N), dtype=np.float32) / np.float32(np.sqrt(N))
    return ((A + A.T) * np.float32(0.5)).astype(dtype)


def paper_upper_gauss(N: int = 16, sigma: float = 10.0, seed: int | None = None, tag: int = 100) -> np.ndarray:
    """Sec 4 / Sec 8.2 generator: upper-triangular Q_ij ~ N(0, sigma^2) for
    i <= j.  Returned as the build's matrix (the paper's Q negated), to be
    used with the UPPER layout and beta = 1."""
    rng = _rng(tag, seed)
    U = np.triu(rng.normal(0.0, sigma, size=(N, N)))
    return -U


def example2() -> np.ndarray:
    """Sec 2.2 Example 2: 16 states on the 4-cube with pi proportional to
    e^{level}; as a QUBO this is N = 4, Q = -I, beta = 1."""
    return -np.eye(4, dtype=np.int32)


def beta_ladder(num: int = 16, lo: float = 0.1, hi: float = 3.0) -> np.ndarray:
    """Geometric inverse-temperature ladder lo .. hi (temperature replicas)."""
    if num == 1:
        return np.array([lo])
    return lo * (hi / lo) ** (np.arange(num) / (num - 1))


@dataclass
class Workload:
    name: str
    Q: np.ndarray | List[np.ndarray]
    betas: np.ndarray
    mode: str
    subset: int
    steps: int
    L0: int = 100
    layout: str = "symmetric"
    extra: dict = field(default_factory=dict)


def c1_basic_n16(seed: int | None = None, chains: int = 1) -> Workload:
    """Basic PNS, dense symmetric int32 QUBO N=16, entries U{-50..50},
    beta = 0.05, subset 4, 2e5 steps."""
    Q = symmetric_int(16, -50, 50, np.int32, seed, tag=1)
    return Workload("basic_n16_int32", Q, np.full(chains, 0.05), "basic", 4, 200_000)


def c2_rf_n1024(seed: int | None = None, mode: str = "rf", chains: int = 1024) -> Workload:
    """Rejection-Free (or Basic PNS subset 64), dense symmetric int16 QUBO
    N=1024, entries U{-100..100}, 1024 chains, beta = 0.01, 1e5 steps."""
    Q = symmetric_int(1024, -100, 100, np.int16, seed, tag=2)
    return Workload(f"{mode}_n1024_int16", Q, np.full(chains, 0.01), mode, 1024 if mode == "rf" else 64, 100_000)


def c3_unbiased_n8192(seed: int | None = None, replicas: int = 256, temps: int = 16) -> Workload:
    """Unbiased PNS (systematic sets), dense float32 QUBO N=8192,
    Q = (A + A^T)/2 with A ~ N(0,1)/sqrt(N), 256 chains x 16 temperatures on
    a geometric ladder 0.1 .. 3.0, subset 512, L0 = 100, 1e5 steps."""
    Q = symmetric_gauss(8192, seed, tag=3)
    betas = np.tile(beta_ladder(temps), replicas)
    return Workload("unbiased_n8192_f32", Q, betas, "unbiased_sys", 512, 100_000)


def c4_batched(seed: int | None = None, problems: int = 64, chains_per: int = 64, only=None) -> Workload:
    """64 int16 QUBOs of uneven N, log-uniform in [256, 16384], entries
    U{-100..100} kept with probability 1/2, 64 chains each, beta scaled as
    0.01 * sqrt(2048 / N) so that beta * std(local field) stays comparable.
    ``only``: generate just these problems' matrices (the others are None)."""
    rng = _rng(4, seed)
    Ns = np.rint(np.exp(rng.uniform(np.log(256), np.log(16384), size=problems))).astype(int)
    Qs = [symmetric_int(int(N), -100, 100, np.int16, seed=SEED_BASE + 4000 + i if seed is None else seed + 4000 + i,
                        density=0.5) if only is None or i in only else None for i, N in enumerate(Ns)]
    betas = np.repeat(0.01 * np.sqrt(2048.0 / Ns), chains_per)
    return Workload("batched_64_uneven_int16", Qs, betas, "unbiased_sys", 0, 100_000,
                    extra={"Ns": Ns, "chains_per": chains_per})


def c5_fit(N: int, seed: int | None = None, chains: int = 8192) -> Workload:
    """Ground-truth float32 QUBO for the maximum-likelihood fit, N in
    {64, 512}, Q* = (A + A^T)/2, A ~ N(0,1)/sqrt(N), beta = 1."""
    Q = symmetric_gauss(N, seed, tag=50 + N)
    return Workload(f"fit_n{N}_f32", Q, np.ones(chains), "rf", N, 0)


def donut_draws(C: int, dim: int = 2, mu0: float = 9.0, sigma: float = 0.1, seed: int | None = None,
                tag: int = 200) -> np.ndarray:
    """C exact draws [C, dim] from the donut density of Sec 7,
    f(x) proportional to exp(-(|x|^2 - mu0)^2 / (2 sigma^2)) on R^dim: the
    squared radius u = |x|^2 has density proportional to
    exp(-(u - mu0)^2 / (2 sigma^2)) u^(dim/2 - 1) on u > 0 (drawn by rejection
    from the normal N(mu0, sigma^2) restricted to mu0 +- 12 sigma, u > 0), and
    the direction is uniform on the sphere (a normalised Gaussian vector)."""
    rng = _rng(tag, seed)
    lo, hi = max(mu0 - 12 * sigma, 1e-12), mu0 + 12 * sigma
    g_max = max(lo ** (dim / 2 - 1), hi ** (dim / 2 - 1))
    u = np.empty(0)
    while u.size < C:
        v = rng.normal(mu0, sigma, size=2 * C)
        v = v[(v > lo) & (v < hi)]
        keep = rng.random(v.size) * g_max < v ** (dim / 2 - 1)
        u = np.concatenate([u, v[keep]])
    g = rng.standard_normal((C, dim))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return np.sqrt(u[:C])[:, None] * g


def donut_ring(C: int, dim: int = 2, mu0: float = 9.0) -> np.ndarray:
    """C states on the ring |x|^2 = mu0 at evenly spaced angles in the
    (x_0, x_1) plane (a deterministic start away from equilibrium in angle)."""
    x = np.zeros((C, dim))
    ang = 2 * np.pi * np.arange(C) / max(C, 1)
    x[:, 0] = np.sqrt(mu0) * np.cos(ang)
    if dim > 1:
        x[:, 1] = np.sqrt(mu0) * np.sin(ang)
    return x
