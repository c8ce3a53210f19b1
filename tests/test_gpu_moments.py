"""GPU parity of the differentiation path: the MFMA moment kernel and the
enumeration of log Z against the oracle, the sampled gradient of LogZ
against exact enumeration and finite differences of log Z (N <= 16), and a
maximum-likelihood fit of a QUBO to synthetic samples."""
import math

import numpy as np
import pytest

from oracle import exact, moments
from paper_2210_10513_amd import inputs

pytestmark = pytest.mark.gpu


def _rand_records(K, N, seed, mmax, density=0.5):
    rng = np.random.default_rng(seed)
    X = (rng.random((K, N)) < density).astype(np.uint8)
    m = rng.integers(0, mmax + 1, size=K).astype(np.int64)
    return X, m


@pytest.mark.parametrize("K,N", [(0, 5), (1, 1), (63, 7), (64, 64), (65, 65), (1000, 100), (5000, 130),
                                 (20000, 512)])
@pytest.mark.parametrize("mmax", [1, 256, 60000, 1 << 18])
def test_moments_exact_against_oracle(K, N, mmax):
    """Exact (integer) equality for weights up to 2^18: one, two and three
    bf16 pieces, ragged K and N, K below one MFMA step."""
    from paper_2210_10513_amd import binding
    X, m = _rand_records(K, N, seed=K + N + mmax, mmax=mmax)
    G = np.full((N, N), -1.0)
    sm = binding.pns_moments(X, m, G)
    want = moments.weighted_moments(X, m)
    assert sm == float(m.sum())
    assert np.array_equal(G, want.astype(np.float64))


def test_moments_large_weights_within_stated_bound():
    """Weights beyond 2^18 (chunks of 64 records): relative error of each
    entry below 64 * 2^-24 plus the 24-bit rounding of each weight."""
    from paper_2210_10513_amd import binding
    X, m = _rand_records(3000, 40, seed=5, mmax=1 << 40)
    G = np.zeros((40, 40))
    binding.pns_moments(X, m, G)
    want = moments.weighted_moments(X, m).astype(np.float64)
    rel = np.abs(G - want) / np.maximum(want, 1.0)
    assert rel.max() <= 64 * 2.0 ** -24 + 2.0 ** -24


def test_moments_device_buffers_and_ldx():
    import torch
    from paper_2210_10513_amd import binding
    K, N, ld = 777, 50, 64
    X, m = _rand_records(K, ld, seed=9, mmax=100)
    Xt = torch.from_numpy(X).cuda()
    mt = torch.from_numpy(m).cuda()
    G = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    binding.pns_moments(Xt, mt, G, N=N, ldx=ld, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), moments.weighted_moments(X[:, :N], m).astype(np.float64))


def test_snapshot_moments_equal_oracle_on_read_back_snapshots():
    from paper_2210_10513_amd.binding import Sampler
    Q = inputs.symmetric_int(90, -30, 30, np.int32, seed=4)
    s = Sampler(Q, 0.05, 0, "rf", num_chains=37, seed=2, init="random", snapshot_every=3, snapshot_capacity=10)
    s.run(40)  # 13 snapshots into a ring of 10
    xs, ms, es, cnt = s.read_snapshots()
    G, sm = s.snapshot_moments()
    s.close()
    assert cnt == 10
    X = xs.reshape(-1, 90)
    m = ms.reshape(-1)
    assert sm == float(m.sum())
    assert np.array_equal(G, moments.weighted_moments(X, m).astype(np.float64))


def test_logz_grad_is_the_scaled_snapshot_moments():
    """pns_logz_grad: -beta * G / sum_w of the snapshots on the device, equal
    bit for bit to the same expression formed from pns_snapshot_moments (and
    _rb) read back to the host; host buffers are rejected."""
    import torch
    from paper_2210_10513_amd import binding as b
    from paper_2210_10513_amd.binding import Sampler
    N, beta = 40, 0.3
    Q = inputs.symmetric_int(N, -20, 20, np.int32, seed=41)
    s = Sampler(Q, beta, 0, "rf", num_chains=64, seed=5, init="random", snapshot_every=3, snapshot_capacity=16)
    s.run(60)
    for rb in (False, True):
        Gd = torch.empty((N, N), dtype=torch.float64, device="cuda")
        sd = torch.empty(1, dtype=torch.float64, device="cuda")
        b.pns_snapshot_moments(s.ctx, 0, Gd, sum_m=sd, rb=rb)
        ref = Gd.cpu().numpy() * (-beta / sd.cpu().numpy()[0])
        gd = torch.empty((N, N), dtype=torch.float64, device="cuda")
        sw = torch.empty(1, dtype=torch.float64, device="cuda")
        b.pns_logz_grad(s.ctx, 0, beta, gd, sw, rb=rb)
        torch.cuda.synchronize()
        assert sw.item() == sd.item()
        assert np.array_equal(gd.cpu().numpy(), ref)
        assert np.allclose(ref, ref.T)
    with pytest.raises(b.PNSError) as ei:
        b.pns_logz_grad(s.ctx, 0, beta, np.zeros((N, N)), np.zeros(1))
    assert ei.value.code == b.PNS_EINVAL
    s.close()


def test_snapshot_moments_before_the_ring_fills():
    from paper_2210_10513_amd.binding import Sampler
    Q = inputs.symmetric_int(20, -30, 30, np.int32, seed=5)
    s = Sampler(Q, 0.1, 0, "rf", num_chains=5, seed=2, snapshot_every=4, snapshot_capacity=8)
    s.run(13)  # 3 of 8 slots written
    xs, ms, _, cnt = s.read_snapshots()
    G, sm = s.snapshot_moments()
    s.close()
    assert cnt == 3
    X = xs[:, :3].reshape(-1, 20)
    m = ms[:, :3].reshape(-1)
    assert sm == float(m.sum())
    assert np.array_equal(G, moments.weighted_moments(X, m).astype(np.float64))


@pytest.mark.parametrize("dtype,layout", [(np.int16, "symmetric"), (np.int32, "upper"), (np.float32, "symmetric"),
                                          (np.float32, "upper")])
@pytest.mark.parametrize("N", [1, 5, 12, 16, 20])
def test_log_partition_against_enumeration(dtype, layout, N):
    from paper_2210_10513_amd import binding
    rng = np.random.default_rng(N)
    if np.issubdtype(dtype, np.integer):
        U = rng.integers(-20, 21, size=(N, N))
    else:
        U = rng.standard_normal((N, N)) * 2
    Q = (np.triu(U) + np.triu(U, 1).T) if layout == "symmetric" else np.triu(U)
    Q = Q.astype(dtype)
    lay = binding.PNS_SYMMETRIC if layout == "symmetric" else binding.PNS_UPPER
    for beta in (0.0, 0.37):
        got = binding.pns_log_partition(Q, beta, layout=lay)
        want = exact.log_partition(Q.astype(np.float64), beta, layout=lay)
        assert math.isclose(got, want, rel_tol=1e-12, abs_tol=1e-12), (got, want)


def test_log_partition_finite_differences_give_second_moments():
    """Central differences of the device log Z in Q_ij equal the oracle's
    -beta E[x_i x_j] (times 2 off the diagonal)."""
    from paper_2210_10513_amd import binding
    N = 10
    rng = np.random.default_rng(3)
    U = rng.standard_normal((N, N))
    Q = ((U + U.T) / 2).astype(np.float32)
    beta = 0.8
    g = moments.grad_log_partition(Q.astype(np.float64), beta)
    eps = 1e-2
    for i, j in [(0, 0), (2, 7), (9, 9), (4, 5)]:
        Dp = Q.astype(np.float64).copy()
        Dm = Q.astype(np.float64).copy()
        Dp[i, j] += eps
        Dm[i, j] -= eps
        if i != j:
            Dp[j, i] += eps
            Dm[j, i] -= eps
        # the step is the float32 difference actually applied to Q_ij
        fd = (binding.pns_log_partition(Dp.astype(np.float32), beta) -
              binding.pns_log_partition(Dm.astype(np.float32), beta)) / (
                 (Dp[i, j].astype(np.float32) - Dm[i, j].astype(np.float32)))
        want = g[i, j] * (2 if i != j else 1)
        assert abs(fd - want) < 5e-4, (i, j, fd, want)


@pytest.mark.parametrize("mode,n", [("rf", 0), ("unbiased_sys", 6)])
def test_logz_gradient_matches_enumeration(mode, n):
    """LogZ forward = exact log Z; its backward (sampled moments on the MFMA
    kernel) = -beta E_pi[x x^T] within the sampling error of 8192 chains x
    32 snapshots."""
    import torch
    from paper_2210_10513_amd.autograd import ChainOptions, LogZ
    N = 12
    rng = np.random.default_rng(12)
    U = rng.standard_normal((N, N))
    Qn = ((U + U.T) / 2).astype(np.float32)
    beta = 0.7
    Q = torch.tensor(Qn, device="cuda", requires_grad=True)
    opts = ChainOptions(num_chains=8192, burn_in=200, samples=32, every=5, mode=mode, subset_size=n, seed=3)
    lz = LogZ.apply(Q, beta, opts)
    lz.backward()
    assert math.isclose(float(lz.item()), exact.log_partition(Qn.astype(np.float64), beta), rel_tol=1e-6)
    want = moments.grad_log_partition(Qn.astype(np.float64), beta)
    got = Q.grad.cpu().numpy().astype(np.float64)
    assert np.abs(got - want).max() < 0.01 * beta, np.abs(got - want).max()
    # the gradient is symmetric and its diagonal is -beta P(x_i = 1) in [-beta, 0]
    assert np.array_equal(got, got.T)
    assert (np.diag(got) <= 0).all() and (np.diag(got) >= -beta).all()


def test_logz_gradient_matches_finite_differences_of_exact_log_z():
    import torch
    from paper_2210_10513_amd.autograd import ChainOptions, LogZ
    N = 16
    Qn = inputs.symmetric_gauss(N, seed=16) * np.float32(2.0)
    beta = 0.5
    Q = torch.tensor(Qn, device="cuda", requires_grad=True)
    LogZ.apply(Q, beta, ChainOptions(num_chains=8192, burn_in=300, samples=32, every=6, seed=5)).backward()
    got = Q.grad.cpu().numpy().astype(np.float64)
    eps = 1e-4
    for i, j in [(0, 0), (3, 11), (15, 15), (7, 8)]:
        Dp = Qn.astype(np.float64).copy()
        Dm = Qn.astype(np.float64).copy()
        Dp[i, j] += eps
        Dm[i, j] -= eps
        if i != j:
            Dp[j, i] += eps
            Dm[j, i] -= eps
        fd = (exact.log_partition(Dp, beta) - exact.log_partition(Dm, beta)) / (2 * eps)
        want = fd / (2 if i != j else 1)
        assert abs(got[i, j] - want) < 0.01 * beta, (i, j, got[i, j], want)


def test_maximum_likelihood_fit_recovers_moments_n16():
    """Fit Q from zero to the exact second moments of a seeded ground truth:
    the negative log-likelihood falls to near its minimum and the model's
    exact moments approach the data's."""
    import torch
    from paper_2210_10513_amd.autograd import ChainOptions, fit_qubo
    N = 16
    Qt = inputs.symmetric_gauss(N, seed=77).astype(np.float64) * 1.5
    beta = 1.0
    D = exact.second_moments(Qt, beta)
    res = fit_qubo(torch.tensor(D, device="cuda"), beta, iters=60, lr=0.5,
                   opts=ChainOptions(num_chains=4096, burn_in=100, samples=16, every=4, seed=11))
    Qf = res.Q.cpu().numpy().astype(np.float64)
    l_start = moments.nll(np.zeros((N, N)), beta, D)[0]
    l_true = moments.nll(Qt, beta, D)[0]
    l_fit = moments.nll(Qf, beta, D)[0]
    assert l_fit < l_start
    assert l_fit - l_true < 0.05 * (l_start - l_true)
    gap = np.abs(exact.second_moments(Qf, beta) - D).max()
    assert gap < 0.05, gap
    assert res.moment_gap[-1] < res.moment_gap[0]


def test_fit_tail_average_reduces_gradient_noise():
    """With exact data moments (N = 16, enumeration) the fit's remaining
    parameter error is the Monte Carlo noise of its gradients: the mean of
    the last 100 of 200 iterates lies closer to the truth than the last
    iterate, and averaging over the last update alone returns the last
    iterate itself (the sampler and the integer-weighted moments are
    deterministic for fixed seeds)."""
    import torch
    from paper_2210_10513_amd.autograd import ChainOptions, fit_qubo
    N = 16
    Qt = inputs.symmetric_gauss(N, seed=77).astype(np.float64) * 1.5
    D = torch.tensor(exact.second_moments(Qt, 1.0), device="cuda")
    kw = dict(iters=200, lr=0.5, opts=ChainOptions(num_chains=4096, burn_in=100, samples=16, every=4, seed=11))
    last = fit_qubo(D, 1.0, **kw)
    one = fit_qubo(D, 1.0, average_from=199, **kw)
    avg = fit_qubo(D, 1.0, average_from=100, **kw)
    assert torch.equal(last.Q, one.Q)
    Qtt = torch.tensor(Qt, dtype=torch.float32, device="cuda")
    rel_last = float((last.Q - Qtt).norm() / Qtt.norm())
    rel_avg = float((avg.Q - Qtt).norm() / Qtt.norm())
    assert rel_avg < 0.7 * rel_last, (rel_avg, rel_last)
    with pytest.raises(ValueError):
        fit_qubo(D, 1.0, average_from=200, **kw)


@pytest.mark.parametrize("N", [64, 512])
def test_fit_workload_gradient_sampled_entries(N):
    """The fit workload's shape (8192 chains, float32 Q): the backward's G
    against the oracle on sampled entries of the read-back snapshots."""
    from paper_2210_10513_amd.binding import Sampler
    w = inputs.c5_fit(N)
    s = Sampler(w.Q, float(w.betas[0]), 0, "rf", num_chains=8192, seed=7, init="random", snapshot_every=4,
                snapshot_capacity=8)
    s.run(64)
    xs, ms, _, cnt = s.read_snapshots()
    G, sm = s.snapshot_moments()
    s.close()
    X = xs.reshape(-1, N)
    m = ms.reshape(-1)
    assert sm == float(m.sum())
    rng = np.random.default_rng(N)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, N, size=(24, 2))] + [(0, 0), (N - 1, N - 1), (0, N - 1)]
    want = moments.weighted_moment_entries(X, m, pairs)
    got = np.array([G[a, b] for a, b in pairs])
    assert np.array_equal(got, want.astype(np.float64))
    assert np.array_equal(G, G.T)


def test_maximum_likelihood_fit_n64_reaches_the_noise_floor():
    """The fit workload at N = 64: data moments from 2^20 weighted samples of
    the seeded ground truth; 300 centered gradient iterations from zero bring
    the sampled moment gap down to about the gap of the truth itself (the
    sampling-noise floor) and the parameters near the truth."""
    import torch
    from paper_2210_10513_amd.autograd import ChainOptions, LogZ, fit_qubo, moments_of_samples
    N = 64
    Qt = torch.tensor(inputs.c5_fit(N).Q, device="cuda")
    D, ns = moments_of_samples(Qt, 1.0, ChainOptions(num_chains=8192, burn_in=8 * N, samples=128, every=16, seed=1))
    assert ns == 1 << 20
    res = fit_qubo(D, 1.0, 300, 0.1, ChainOptions(num_chains=8192, burn_in=64, samples=16, every=8, seed=3,
                                                  exact_max=0))
    Qg = Qt.clone().requires_grad_(True)
    LogZ.apply(Qg, 1.0, ChainOptions(num_chains=8192, burn_in=8 * N, samples=16, every=8, seed=5,
                                     exact_max=0)).backward()
    floor = float((D.float() + Qg.grad).abs().max())
    gap = float(np.mean(res.moment_gap[-50:]))
    rel = float((res.Q - Qt).norm() / Qt.norm())
    assert res.moment_gap[0] > 10 * floor
    assert gap < 2.0 * floor, (gap, floor)
    assert rel < 0.2, rel
