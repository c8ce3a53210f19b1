"""GPU tests of the window kernel of one, two or four waves per chain
(flavour 5: Unbiased PNS with systematic sets on integer Q): every record
replayed through the oracle on ragged sizes of each of its tiles, the same
records as the step kernel's window flavours on the same problem, the paths
past the weight tables and of a rescaled window, the uninstrumented kernel
against the instrumented one, and a checkpoint resume."""
import numpy as np
import pytest

from paper_2210_10513_amd import inputs

from parity_util import gpu_run, replay_check

pytestmark = pytest.mark.gpu


def _replay(Q, beta, K, *, chains, n, L0, seed, tile, layout="symmetric", init="random", rows=None):
    g = gpu_run(Q, beta, "unbiased_sys", K, chains=chains, n=n, L0=L0, seed=seed, init=init, layout=layout,
                block=tile[0], groups=tile[1])
    assert g["tile"] == tile and g["flavour"] == 5
    rows = list(range(chains)) if rows is None else rows
    b = np.asarray(beta)[rows] if np.ndim(beta) else beta
    _, cov = replay_check(g["log"], Q, b, "unbiased_sys", rows=rows, is_int=True, gcur=g["cur"], n=n, L0=L0,
                          seed=seed, init=init, layout=layout)
    assert cov.compared == len(rows) * K and cov.finals == len(rows)
    assert (g["stats"]["anomalies"] == 0).all()
    return g


@pytest.mark.parametrize("N,n,tile,dtype,layout", [
    (300, 64, (64, 2), np.int16, "symmetric"),      # 512-bit tile: ragged, windows wrap
    (449, 100, (64, 2), np.int32, "upper"),
    (700, 100, (64, 4), np.int32, "symmetric"),     # one wave, four groups, one state word
    (1000, 128, (64, 4), np.int16, "symmetric"),
    (1000, 64, (64, 8), np.int16, "symmetric"),     # ragged last segment, windows wrap
    (700, 100, (64, 8), np.int32, "symmetric"),     # n not a power of two, idle groups
    (2047, 128, (64, 8), np.int32, "upper"),
    (3000, 256, (64, 16), np.int16, "symmetric"),
    (5000, 512, (64, 24), np.int16, "symmetric"),
    (6001, 256, (128, 16), np.int16, "upper"),      # two waves
    (9000, 512, (128, 24), np.int32, "symmetric"),
    (15000, 256, (256, 16), np.int16, "symmetric"),  # four waves
])
def test_window_kernel_replays_against_oracle(N, n, tile, dtype, layout):
    if layout == "upper":
        rng = np.random.default_rng(N)
        Q = np.triu(rng.integers(-100, 101, size=(N, N))).astype(dtype)
    else:
        Q = inputs.symmetric_int(N, -100, 100, dtype, seed=N + n, density=0.5)
    _replay(Q, 0.01 * np.sqrt(2048.0 / N), 300, chains=3, n=n, L0=40, seed=17, tile=tile, layout=layout)


@pytest.mark.parametrize("N,n,step_tile,wave_tile", [(500, 64, (128, 1), (64, 2)),
                                                     (900, 128, (256, 1), (64, 4)),
                                                     (3000, 256, (256, 4), (64, 16)),
                                                     (1500, 128, (128, 4), (64, 8)),
                                                     (7000, 512, (256, 8), (128, 16)),
                                                     (12000, 256, (1024, 4), (128, 24))])
def test_window_kernel_equals_step_kernel(N, n, step_tile, wave_tile):
    """The window kernel sums, scans and chooses in the step kernel's order:
    on the same problem its records (action, M, E, p) and final state equal
    the step kernel's window flavours bit for bit."""
    Q = inputs.symmetric_int(N, -100, 100, np.int16, seed=N, density=0.5)
    beta = 0.01 * np.sqrt(2048.0 / N)
    kw = dict(chains=4, n=n, L0=100, seed=5, init="random")
    a = gpu_run(Q, beta, "unbiased_sys", 400, block=step_tile[0], groups=step_tile[1], **kw)
    b = gpu_run(Q, beta, "unbiased_sys", 400, block=wave_tile[0], groups=wave_tile[1], **kw)
    assert a["flavour"] in (1, 3, 4) and b["flavour"] == 5
    for key in ("action", "M", "E", "p"):
        assert np.array_equal(a["log"][key], b["log"][key]), key
    for key in ("x", "h", "E", "step"):
        assert np.array_equal(a["cur"][key], b["cur"][key]), key


@pytest.mark.parametrize("tile", [(64, 8), (128, 16)])
def test_window_kernel_past_the_tables_and_rescaled(tile):
    """int16 entries up to 30000: most energy differences exceed the 2^16
    range of the tables and their weights come from the exponential (beta =
    2e-6 keeps them between 1e-3 and 1); then a chain whose window weights
    all underflow (large positive diagonal, beta = 3) takes the rescaled
    path.  Every record replays through the oracle."""
    N = 1500 if tile == (64, 8) else 5000
    Q = inputs.symmetric_int(N, -30000, 30000, np.int16, seed=N)
    _replay(Q, 2e-6, 300, chains=3, n=128, L0=40, seed=9, tile=tile)
    D = inputs.symmetric_int(N, -10, 10, np.int16, seed=N + 1)
    np.fill_diagonal(D, 3000)
    _replay(D, 3.0, 200, chains=2, n=128, L0=40, seed=10, tile=tile, init="zero")


@pytest.mark.parametrize("tile,N,n", [((64, 16), 4000, 256), ((256, 16), 16384, 512)])
def test_uninstrumented_window_kernel_equals_instrumented(tile, N, n):
    """The kernel without per-step outputs (the one the benchmark times)
    reaches the same states, fields, energies, last record and counters as
    the instrumented one, whose every record replays through the oracle,
    across two launches."""
    from paper_2210_10513_amd.binding import Sampler
    Q = inputs.symmetric_int(N, -100, 100, np.int16, seed=N, density=0.5)
    beta = 0.01 * np.sqrt(2048.0 / N)
    out = []
    for log in (0, 700):
        s = Sampler(Q, beta, n, "unbiased_sys", num_chains=64, seed=3, init="random", L0=100, block=tile[0],
                    groups=tile[1], log_capacity=log)
        s.run(350)
        s.run(350)
        out.append((s.read_current(), s.read(), s.stats(), s.read_log() if log else None))
        s.close()
    (cu, ru, su, _), (ci, ri, si, li) = out
    for key in ("x", "h", "E", "step"):
        assert np.array_equal(cu[key], ci[key]), key
    for a, b in zip(ru, ri):
        assert np.array_equal(a, b)
    for key in su:
        assert np.array_equal(su[key], si[key]), key
    rows = [0, 31, 63]
    _, cov = replay_check(li, Q, beta, "unbiased_sys", rows=rows, is_int=True, gcur=ci, n=n, L0=100, seed=3,
                          init="random")
    assert cov.compared == len(rows) * 700


def test_window_kernel_checkpoint_resume():
    """Run 2K equals run K, save, load into a fresh context, run K."""
    from paper_2210_10513_amd.binding import Sampler
    Q = inputs.symmetric_int(3000, -100, 100, np.int16, seed=4, density=0.5)
    kw = dict(num_chains=8, seed=6, init="random", L0=50, block=64, groups=16, log_capacity=400)
    a = Sampler(Q, 0.01, 256, "unbiased_sys", **kw)
    a.run(400)
    ref = a.read_log()
    cur = a.read_current()
    a.close()
    b = Sampler(Q, 0.01, 256, "unbiased_sys", **kw)
    b.run(200)
    buf = b.save()
    b.close()
    c = Sampler(Q, 0.01, 256, "unbiased_sys", **kw)
    c.load(buf)
    c.run(200)
    got = c.read_log()
    cur2 = c.read_current()
    c.close()
    for key in ("action", "M", "E"):
        assert np.array_equal(ref[key][:, 200:], got[key][:, 200:]), key
    for key in ("x", "h", "E", "step"):
        assert np.array_equal(cur[key], cur2[key]), key
