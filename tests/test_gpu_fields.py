"""GPU tests of the local fields computed as one matrix product per problem
(H = X A on the int8 matrix cores for integer Q, split into bytes; on the
FP64 matrix cores for float Q): on creation with random or given states,
after pns_set_q, and by pns_refresh, against the exact products computed
here with numpy (int64 / FP64), on ragged N and chain counts around the
64 x 64 tiles, every field type, the upper-triangular layout and a batch."""
import numpy as np
import pytest

from paper_2210_10513_amd import inputs

pytestmark = pytest.mark.gpu


def _offdiag(Q, layout):
    Qs = np.triu(Q) + np.triu(Q, 1).T if layout == "upper" else Q
    A = Qs.copy()
    np.fill_diagonal(A, 0)
    return Qs, A


def _exact(Q, x, layout="symmetric"):
    """Fields h = sum_{j != i} c_ij x_j / s (s = 2 symmetric: h_i = sum Q_ij x_j;
    upper: the pair coefficient) and energies x^T Q x, exactly (int64) or in
    FP64 (float Q)."""
    is_int = np.issubdtype(Q.dtype, np.integer)
    Qw = Q.astype(np.int64 if is_int else np.float64)
    Qs, A = _offdiag(Qw, layout)
    X = x.astype(np.int64 if is_int else np.float64)
    H = X @ A
    if layout == "upper":
        E = np.einsum("ci,ij,cj->c", X, np.triu(Qw), X)
    else:
        E = np.einsum("ci,ij,cj->c", X, Qw, X)
    return H, E


def _check(cur, Q, layout="symmetric"):
    x, h, E = cur["x"], cur["h"], cur["E"]
    H, Er = _exact(Q, x, layout)
    if np.issubdtype(Q.dtype, np.integer):
        assert np.array_equal(h.astype(np.int64), H), "fields differ"
        assert np.array_equal(E, Er.astype(np.float64)), "energies differ"
    else:
        scale = np.maximum(1.0, np.abs(H).max())
        assert np.abs(h - H).max() <= 1e-12 * scale, np.abs(h - H).max()
        assert np.allclose(E, Er, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N", [1, 5, 63, 64, 65, 700, 3000])
@pytest.mark.parametrize("kind", ["i16", "i32", "i32wide", "f32"])
def test_initial_fields_are_the_matrix_product(N, kind):
    from paper_2210_10513_amd.binding import Sampler, pns_field_type
    if kind == "i16":
        Q = inputs.symmetric_int(N, -32000, 32000, np.int16, seed=N)
    elif kind == "i32":
        Q = inputs.symmetric_int(N, -100000, 100000, np.int32, seed=N)
    elif kind == "i32wide":
        Q = inputs.symmetric_int(N, -2_000_000_000, 2_000_000_000, np.int32, seed=N)
    else:
        Q = inputs.symmetric_gauss(N, seed=N) * np.float32(100.0)
    for chains in (1, 17, 70):
        s = Sampler(Q, 1e-9, 0, "rf", num_chains=chains, seed=N + chains, init="random")
        if kind == "i32wide" and N > 1:
            assert pns_field_type(s.ctx) == 1  # int64 fields
        _check(s.read_current(), Q)
        s.close()


def test_given_states_upper_layout_and_batch():
    from paper_2210_10513_amd.binding import BatchSampler, Sampler
    rng = np.random.default_rng(3)
    U = np.triu(rng.integers(-30000, 30001, size=(333, 333))).astype(np.int32)
    x0 = rng.integers(0, 2, size=(9, 333)).astype(np.uint8)
    s = Sampler(U, 1e-9, 0, "rf", num_chains=9, x0=x0, layout="upper")
    cur = s.read_current()
    assert np.array_equal(cur["x"], x0)
    _check(cur, U, "upper")
    s.close()
    probs = [{"Q": inputs.symmetric_int(N, -100, 100, np.int16, seed=N, density=0.5), "num_chains": c, "beta": 0.01,
              "subset_size": 16} for N, c in ((50, 3), (700, 65), (2100, 2), (6000, 5), (12000, 4))]
    b = BatchSampler(probs, "unbiased_sys", seed=4, init="random")
    cur = b.read_current()
    for p, pr in enumerate(probs):
        _check({k: cur[k][p] for k in ("x", "h", "E")}, pr["Q"])
    b.close()


@pytest.mark.parametrize("kind", ["i16", "f32"])
def test_refresh_after_a_long_run(kind):
    """After 3000 steps the refreshed fields equal the incrementally kept ones
    (exactly for integer Q, to FP64 rounding for float Q), the last record is
    kept, and the chains continue."""
    from paper_2210_10513_amd.binding import Sampler
    N = 1500
    if kind == "i16":
        Q, beta = inputs.symmetric_int(N, -100, 100, np.int16, seed=5), 0.01
    else:
        Q, beta = inputs.symmetric_gauss(N, seed=5), 1.0
    s = Sampler(Q, beta, 100, "unbiased_sys", num_chains=70, seed=8, init="random")
    s.run(3000)
    before, rec = s.read_current(), s.read()
    s.refresh()
    after = s.read_current()
    _check(after, Q)
    assert np.array_equal(before["x"], after["x"]) and np.array_equal(before["step"], after["step"])
    if kind == "i16":
        assert np.array_equal(before["h"], after["h"]) and np.array_equal(before["E"], after["E"])
    else:
        assert np.abs(before["h"] - after["h"]).max() <= 1e-12 * np.abs(after["h"]).max()
    for a, b in zip(rec, s.read()):
        assert np.array_equal(a, b)
    s.run(100)
    assert (s.read_current()["step"] == 3100).all()
    _check(s.read_current(), Q)
    s.close()


def test_set_q_fields_are_the_new_product():
    from paper_2210_10513_amd.binding import Sampler
    Q1 = inputs.symmetric_gauss(512, seed=1)
    Q2 = inputs.symmetric_gauss(512, seed=2)
    s = Sampler(Q1, 1.0, 0, "rf", num_chains=130, seed=3, init="random")
    s.run(200)
    s.set_q(Q2)
    _check(s.read_current(), Q2)
    s.close()
