"""GPU test of pns_moments_noalloc (the moment matrix without allocation,
its workspace a static array per GPU) against pns_moments, through the C ABI:
two calls in a row, the second with a smaller input (the workspace keeps the
first call's contents), bit-exact for integer weights; plus the refusals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(K, N, ldx, seed, mmax):
    import torch
    rng = np.random.default_rng(seed)
    X = torch.from_numpy((rng.random((K, ldx)) < 0.4).astype(np.uint8)).cuda()
    m = torch.from_numpy(rng.integers(0, mmax, size=K).astype(np.int64)).cuda()
    return X, m


def _both(X, m, N):
    import torch
    from paper_2210_10513_amd import binding as b
    G0 = torch.full((N, N), 7.0, dtype=torch.float64, device="cuda")  # overwritten
    s0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    b.pns_moments(X, m, G0, N=N, sum_m=s0)
    G1 = torch.full((N, N), -3.0, dtype=torch.float64, device="cuda")
    s1 = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    b.pns_moments_noalloc(X, m, G1, s1, N=N)
    torch.cuda.synchronize()
    return G0.cpu().numpy(), s0.item(), G1.cpu().numpy(), s1.item()


def test_noalloc_moments_equal_the_allocating_entry_point_twice():
    """First the fit shape (K = 131072 snapshot records, N = 512), then a
    smaller ragged input: both equal pns_moments bit for bit, and the second
    is unaffected by what the first left in the workspace."""
    for K, N, ldx, seed in ((131072, 512, 512, 1), (1000, 77, 80, 2)):
        X, m = _inputs(K, N, ldx, seed, 1 << 16)
        G0, s0, G1, s1 = _both(X, m, N)
        assert np.array_equal(G0, G1), (K, N)
        assert s0 == s1 == float(m.sum().item())
        # and against the definition on sampled entries
        Xn, mn = X.cpu().numpy()[:, :N].astype(np.int64), m.cpu().numpy()
        for i, j in ((0, 0), (N - 1, 3), (5, N - 1)):
            assert G1[i, j] == float((mn * Xn[:, i] * Xn[:, j]).sum())


def test_noalloc_refuses_host_buffers_and_oversized_inputs():
    import torch
    from paper_2210_10513_amd import binding as b
    X, m = _inputs(64, 16, 16, 3, 10)
    G = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(b.PNSError) as ei:
        b.pns_moments_noalloc(X.cpu().numpy(), m, G)
    assert ei.value.code == b.PNS_EINVAL and "device memory" in str(ei.value)
    # 2^20 records of N = 1024: 128 MiB of packed records, beyond the workspace
    Xbig = torch.zeros((1 << 20, 1024), dtype=torch.uint8, device="cuda")
    mbig = torch.ones(1 << 20, dtype=torch.int64, device="cuda")
    Gbig = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    with pytest.raises(b.PNSError) as ei:
        b.pns_moments_noalloc(Xbig, mbig, Gbig)
    assert ei.value.code == b.PNS_EINVAL and "workspace" in str(ei.value)
    # a refused call leaves the next one correct
    G0, s0, G1, s1 = _both(X, m, 16)
    assert np.array_equal(G0, G1) and s0 == s1
