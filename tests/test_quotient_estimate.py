"""Error bounds behind the step kernel's estimate of q = log U1 / log1p(-p)
(the quotient whose floor is the multiplicity and whose order against the
budget L decides a stay, Alg 6).  The kernel estimates log1p(-p) from its
series -p (1 + p/2 + p^2/3 + p^3/4) for p <= 2^-6 and from the float32
logarithm of 1 - p above, and trusts the estimate only when q (1 -+ d)
brackets neither L nor an integer, d = 1e-7 after the series and 1e-4 after
the float logarithm.  These checks restate the two estimates in numpy and
confirm, on a dense grid of p, that their relative errors stay well below the
brackets (series < 1.3e-8, float logarithm < 5e-6), so the bracket rule can
only pick the exact quotient's floor and side of L.  CPU only."""
import numpy as np

D_SERIES, D_LOG = 1e-7, 1e-4


def _series(p):
    return -p * (1.0 + p * (0.5 + p * (1.0 / 3.0 + p * 0.25)))


def _float_log(p):
    return np.log((1.0 - p).astype(np.float32)).astype(np.float64)


def test_series_branch_error():
    p = np.concatenate([np.geomspace(1e-300, 2.0 ** -6, 20001), [2.0 ** -6]])
    exact = np.log1p(-p)
    rel = np.abs(_series(p) - exact) / np.abs(exact)
    assert rel.max() < 1.3e-8, rel.max()
    assert rel.max() < D_SERIES / 7


def test_float_log_branch_error():
    # from just above 2^-6 to 1 - 2^-100 (closer to 1 the kernel computes exactly)
    p = np.concatenate([np.linspace(2.0 ** -6, 0.999, 200001), 1.0 - np.geomspace(1e-3, 2.0 ** -100, 20001)])
    p = p[(p > 2.0 ** -6) & (1.0 - p >= 2.0 ** -100)]
    exact = np.log1p(-p)
    rel = np.abs(_float_log(p) - exact) / np.abs(exact)
    assert rel.max() < 5e-6, rel.max()
    assert rel.max() < D_LOG / 20


def test_bracket_rule_reproduces_floor_and_budget_side():
    """On random (U1, p, L) the bracket rule, applied to the estimate, returns
    the exact floor and the exact side of L whenever it accepts."""
    rng = np.random.default_rng(5)
    n = 200000
    logu = np.log((rng.integers(0, 2 ** 53, n) + 1) * 2.0 ** -53)
    p = np.exp(rng.uniform(np.log(1e-6), np.log(0.999), n))
    L = rng.integers(0, 200, n).astype(np.float64)
    series = p <= 2.0 ** -6
    l1p = np.where(series, _series(p), _float_log(p))
    d = np.where(series, D_SERIES, D_LOG)
    qe = logu / l1p
    q = logu / np.log1p(-p)
    lo, hi = qe * (1 - d), qe * (1 + d)
    accept = (qe < 2.0 ** 52) & (np.floor(lo) == np.floor(hi)) & ~((lo < L) & (hi >= L))
    assert accept.mean() > 0.97
    assert np.array_equal(np.floor(qe[accept]), np.floor(q[accept]))
    assert np.array_equal(qe[accept] >= L[accept], q[accept] >= L[accept])
