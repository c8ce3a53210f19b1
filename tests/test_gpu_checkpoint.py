"""GPU tests of checkpoints (pns_save / pns_load): K steps, save, load into a
freshly created context, K more steps must give bit for bit what one run of
2K steps gives (records, states, fields, energies, counters), in every mode
and for batches, tempering ladders and optimization runs; and bad
checkpoints are refused without touching the context."""
import numpy as np
import pytest

from paper_2210_10513_amd import inputs

pytestmark = pytest.mark.gpu


def _same(a, b, keys):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("mode,n,dtype", [("rf", 0, np.int16), ("basic", 9, np.int32),
                                          ("unbiased_sys", 21, np.int16), ("unbiased_rand", 17, np.int32),
                                          ("unbiased_sys", 40, np.float32), ("rf", 0, np.float32)])
@pytest.mark.parametrize("log", [True, False])
def test_resume_equals_one_run(mode, n, dtype, log):
    from paper_2210_10513_amd.binding import Sampler
    N, C, K = 333, 5, 240
    Q = inputs.symmetric_int(N, -60, 60, dtype, seed=N + n) if dtype != np.float32 else \
        inputs.symmetric_gauss(N, seed=N + n)
    beta = 0.04 if dtype != np.float32 else 1.5
    kw = dict(num_chains=C, L0=30, seed=77, init="random")
    full = Sampler(Q, beta, n, mode, log_capacity=2 * K if log else 0, **kw)
    full.run(2 * K)
    a = Sampler(Q, beta, n, mode, log_capacity=K if log else 0, **kw)
    a.run(K)
    ck = a.save()
    a.close()
    b = Sampler(Q, beta, n, mode, log_capacity=K if log else 0, **kw)
    b.load(ck)
    b.run(K)
    for x, y in zip(full.read(), b.read()):
        assert np.array_equal(x, y)
    _same(full.read_current(), b.read_current(), ("x", "h", "E", "L", "sub", "step"))
    _same(full.stats(), b.stats(), ("steps", "flips", "stays", "saturated", "sum_M", "anomalies"))
    if log:
        lf, lb = full.read_log(), b.read_log()
        for k in ("action", "M", "E", "p"):
            assert np.array_equal(lf[k][:, K:], lb[k]), k
    full.close()
    b.close()


def test_resume_batch_of_uneven_problems_on_device_buffer():
    """A batch (three tiles, random sets in memory), checkpoint in a device
    buffer, graph launch form after the load."""
    import torch
    from paper_2210_10513_amd import binding as bd
    from paper_2210_10513_amd.binding import BatchSampler
    probs = []
    for i, N in enumerate((40, 300, 1100)):
        probs.append({"Q": inputs.symmetric_int(N, -50, 50, np.int16, seed=90 + i), "num_chains": 3,
                      "beta": 0.03, "subset_size": 16 + 8 * i})
    K = 150
    full = BatchSampler(probs, "unbiased_rand", L0=20, seed=5)
    full.run(2 * K)
    a = BatchSampler(probs, "unbiased_rand", L0=20, seed=5)
    a.run(K)
    size = bd.pns_save(a.ctx)
    dbuf = torch.zeros(size, dtype=torch.uint8, device="cuda")
    assert bd.pns_save(a.ctx, dbuf) == size
    a.close()
    b = BatchSampler(probs, "unbiased_rand", L0=20, seed=5, launch="graph", chunk=50)
    bd.pns_load(b.ctx, dbuf, size)
    b.run(K)
    cf, cb = full.read_current(), b.read_current()
    for k in ("x", "h", "E", "L", "sub", "step"):
        for p in range(3):
            assert np.array_equal(cf[k][p], cb[k][p]), (k, p)
    sf, sb = full.stats(), b.stats()
    for k in ("steps", "flips", "stays", "sum_M"):
        assert np.array_equal(sf[k], sb[k]), k
    full.close()
    b.close()


def test_resume_keeps_tempering_ladder_and_best_states():
    from paper_2210_10513_amd.binding import Sampler
    N, T, groups = 40, 4, 8
    C = T * groups
    Q = inputs.symmetric_int(N, -20, 20, np.int32, seed=9)
    betas = np.tile(inputs.beta_ladder(T, 0.02, 0.5), groups)

    def sweeps(s, r0, r1):
        for r in range(r0, r1):
            s.run_original(7)
            s.pt_swap(T, r)

    full = Sampler(Q, betas, 0, "rf", num_chains=C, seed=13, init="random")
    full.optimize(50, 0.7)
    sweeps(full, 0, 12)
    a = Sampler(Q, betas, 0, "rf", num_chains=C, seed=13, init="random")
    a.optimize(50, 0.7)
    sweeps(a, 0, 6)
    ck = a.save()
    a.close()
    b = Sampler(Q, betas, 0, "rf", num_chains=C, seed=13, init="random")
    b.load(ck)
    sweeps(b, 6, 12)
    assert np.array_equal(full.betas(), b.betas()) and np.array_equal(full.ladder(), b.ladder())
    for x, y in zip(full.read_best(), b.read_best()):
        assert np.array_equal(x, y)
    _same(full.read_current(), b.read_current(), ("x", "h", "E", "step"))
    full.close()
    b.close()


def test_bad_checkpoints_are_refused_and_change_nothing():
    from paper_2210_10513_amd.binding import PNSError, Sampler
    Q = inputs.symmetric_int(64, -30, 30, np.int32, seed=2)
    a = Sampler(Q, 0.05, 8, "unbiased_sys", num_chains=3, seed=1)
    a.run(50)
    ck = a.save()
    b = Sampler(Q, 0.05, 8, "unbiased_sys", num_chains=3, seed=1)
    b.run(10)
    before = b.read_current()
    bad = ck.copy()
    bad[len(bad) // 2] ^= 0xFF
    others = [Sampler(Q, 0.05, 8, "unbiased_sys", num_chains=4, seed=1),           # chain count
              Sampler(Q, 0.05, 9, "unbiased_sys", num_chains=3, seed=1),           # subset size
              Sampler(Q, 0.05, 8, "unbiased_sys", num_chains=3, seed=2),           # seed
              Sampler(Q, 0.05, 8, "unbiased_rand", num_chains=3, seed=1),          # mode
              Sampler(Q, 0.05, 8, "unbiased_sys", num_chains=3, seed=1, chain_id_base=5)]
    for blob, ctx in [(bad, b), (ck[:-1], b), (ck[:100], b)] + [(ck, o) for o in others]:
        with pytest.raises(PNSError):
            ctx.load(blob)
    _same(before, b.read_current(), ("x", "h", "E", "L", "sub", "step"))
    b.load(ck)
    _same(a.read_current(), b.read_current(), ("x", "h", "E", "L", "sub", "step"))
    for s in [a, b] + others:
        s.close()
