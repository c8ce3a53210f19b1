"""Pins for the CPU oracle: each test checks the oracle against something the
paper or the mathematics fixes (published test vectors, the paper's worked
examples, brute-force enumeration, closed forms, special cases), never
against a retyping of the oracle's own formula.  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2210_10513_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_json(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _small_int_q(N, seed, lo=-50, hi=50):
    return inputs.symmetric_int(N, lo, hi, np.int64, seed=seed)


def _states_from_actions(x0, actions):
    """Record states J_0 .. J_{K-1} of one chain rebuilt from its actions."""
    x = np.array(x0, dtype=np.uint8)
    out = np.empty((len(actions), len(x)), dtype=np.uint8)
    for k, a in enumerate(actions):
        out[k] = x
        if a >= 0:
            x[a] ^= 1
    return out, x


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_uniforms_ranges_and_moments():
    u1 = np.array([oracle.uniforms(11, c, k)[0] for c in range(20) for k in range(500)])
    u2 = np.array([oracle.uniforms(11, c, k)[1] for c in range(20) for k in range(500)])
    assert u1.min() > 0.0 and u1.max() <= 1.0
    assert u2.min() >= 0.0 and u2.max() < 1.0
    for u in (u1, u2):
        assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
        assert abs((u ** 2).mean() - 1 / 3) < 0.01


def test_random_subset_exact_size_and_uniform():
    N, n, T = 20, 5, 6000
    counts = np.zeros(N)
    pair = np.zeros((N, N))
    for k in range(T):
        m = oracle.random_subset(3, 1, k, N, n)
        assert m.sum() == n
        counts += m
        mi = m.astype(float)
        pair += np.outer(mi, mi)
    # inclusion probability n/N for each index (chi-square, N-1 dof)
    exp_c = T * n / N
    chi2 = ((counts - exp_c) ** 2 / exp_c).sum()
    assert chi2 < 55  # 99.99% quantile of chi2(19) is ~ 50.8
    # pairwise inclusion n(n-1)/(N(N-1)) (uniform n-subset, not independent bits)
    off = pair[~np.eye(N, dtype=bool)] / T
    assert abs(off.mean() - n * (n - 1) / (N * (N - 1))) < 0.003
    # n == N takes everything
    assert oracle.random_subset(3, 1, 0, N, N).all()


def test_random_state_bernoulli_half():
    x = np.concatenate([oracle.random_state(5, c, 257) for c in range(40)])
    assert abs(x.mean() - 0.5) < 4 * 0.5 / np.sqrt(len(x))


# --------------------------------------------------------------------------
# Partial neighbor sets
# --------------------------------------------------------------------------

def test_systematic_sets_match_the_sec5_example():
    g = _golden_json("paper_examples.json")["systematic_sets"]
    N, n = g["N"], g["n"]
    assert oracle.sys_count(N, n) == g["count"]
    for i, bits in enumerate(g["first_three_one_indexed"]):
        m = oracle.sys_subset(N, n, i)
        assert sorted(np.nonzero(m)[0] + 1) == sorted(bits)
    # the schedule is periodic with the stated number of sets and covers all bits
    cover = np.zeros(N, dtype=bool)
    for i in range(g["count"]):
        cover |= oracle.sys_subset(N, n, i)
    assert cover.all()
    assert (oracle.sys_subset(N, n, g["count"]) == oracle.sys_subset(N, n, 0)).all()


def test_systematic_halves():
    N = _golden_json("paper_examples.json")["halves"]["N"]
    assert oracle.sys_count(N, N // 2) == 2
    assert (np.nonzero(oracle.sys_subset(N, N // 2, 0))[0] == np.arange(N // 2)).all()
    assert (np.nonzero(oracle.sys_subset(N, N // 2, 1))[0] == np.arange(N // 2, N)).all()


# --------------------------------------------------------------------------
# Energies, local fields and the recorded trajectory
# --------------------------------------------------------------------------

def test_energy_matches_matrix_product_and_layouts():
    rng = np.random.default_rng(0)
    N = 9
    Q = _small_int_q(N, 4)
    U = np.triu(Q) + np.triu(Q, 1)  # upper-triangular form of the same quadratic form
    E_sym = oracle.enumerate_energies(Q, oracle.LAYOUT_SYMMETRIC)
    E_up = oracle.enumerate_energies(U, oracle.LAYOUT_UPPER)
    X = ((np.arange(1 << N)[:, None] >> np.arange(N)[None, :]) & 1).astype(np.int64)
    E_mat = np.einsum("si,ij,sj->s", X, Q, X)
    assert (E_sym == E_mat).all() and (E_up == E_mat).all()
    Qf = rng.standard_normal((N, N))
    Qf = (Qf + Qf.T) / 2
    Ef = oracle.enumerate_energies(Qf, oracle.LAYOUT_SYMMETRIC)
    assert np.allclose(Ef, np.einsum("si,ij,sj->s", X, Qf, X), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode,n", [(oracle.MODE_RF, 0), (oracle.MODE_BASIC, 3), (oracle.MODE_UNBIASED_SYS, 4),
                                    (oracle.MODE_UNBIASED_RAND, 5)])
@pytest.mark.parametrize("kind", ["int_sym", "int_upper", "float_sym"])
def test_trajectory_energies_and_fields(mode, n, kind):
    """Every record's energy equals x^T Q x of the record's state (brute force
    with a matrix product), every move is a single-bit flip inside the
    declared subset rules, and the final local fields equal the off-diagonal
    matrix-vector product."""
    N, K = 10, 600
    rng = np.random.default_rng(1)
    if kind == "float_sym":
        A = rng.standard_normal((N, N))
        Q = (A + A.T) / 2
        layout = oracle.LAYOUT_SYMMETRIC
        Qsym = Q
    elif kind == "int_sym":
        Q = _small_int_q(N, 2)
        layout = oracle.LAYOUT_SYMMETRIC
        Qsym = Q.astype(np.float64)
    else:
        Q = np.triu(_small_int_q(N, 3))
        layout = oracle.LAYOUT_UPPER
        Qsym = (Q + Q.T) / 2.0
    r = oracle.run(Q, 0.05, mode, K, n=n, L0=7, seed=9, num_chains=3, init="random", layout=layout)
    for c in range(3):
        x0 = oracle.random_state(9, c, N)
        states, xf = _states_from_actions(x0, r.action[c])
        E_bf = np.einsum("si,ij,sj->s", states.astype(float), Qsym, states.astype(float))
        assert np.allclose(r.E[c], E_bf, rtol=1e-12, atol=1e-9)
        assert (r.x[c] == xf).all()
        E_final = xf.astype(float) @ Qsym @ xf.astype(float)
        assert np.isclose(float(r.E_final[c]), E_final, rtol=1e-12, atol=1e-9)
        off = Qsym - np.diag(np.diag(Qsym))
        scale = 2.0 if layout == oracle.LAYOUT_SYMMETRIC else 1.0
        h_expect = (2.0 / scale) * (off @ xf.astype(float))
        assert np.allclose(r.h[c].astype(float), h_expect, rtol=1e-12, atol=1e-9)
        # energy differences of the flips equal brute-force E(x ^ e_c) - E(x)
        moves = np.nonzero(r.action[c] >= 0)[0][:-1]
        assert np.allclose(np.diff(r.E[c].astype(float))[moves], (E_bf[moves + 1] - E_bf[moves]), atol=1e-9)
        if mode == oracle.MODE_UNBIASED_SYS:
            # every flip stays inside the set in force at that step
            sub = 0
            for k, a in enumerate(r.action[c]):
                if a == oracle.STAY:
                    sub += 1
                else:
                    assert oracle.sys_subset(N, n, sub % oracle.sys_count(N, n))[a]
        if mode == oracle.MODE_BASIC:
            for k, a in enumerate(r.action[c][:50]):
                assert oracle.random_subset(9, c, k, N, n)[a]
    if kind.startswith("int"):
        assert r.E.dtype == np.int64


# --------------------------------------------------------------------------
# Multiplicities
# --------------------------------------------------------------------------

def test_multiplicity_is_one_plus_geometric():
    """M | p ~ 1 + Geometric(p) counting failures (Sec 1.2, eq. (2) and the
    jump-chain example): E[p M] = 1, P(M = 1) = p, and M = 1 whenever p = 1."""
    Q = _small_int_q(12, 7, -20, 20)
    r = oracle.run(Q, 0.05, oracle.MODE_RF, 20000, seed=3, num_chains=8)
    p = r.p.ravel()
    M = r.M.ravel().astype(float)
    assert (M >= 1).all()
    assert (M[p == 1.0] == 1).all()
    k = len(p)
    z1 = (p * M).mean() - 1.0
    assert abs(z1) < 5 * np.sqrt(np.mean(1 - p) / k) + 1e-12
    z2 = ((M == 1).astype(float) - p).mean()
    assert abs(z2) < 5 * np.sqrt(np.mean(p * (1 - p)) / k) + 1e-12
    # the geometric tail: P(M > m | p) = (1-p)^m, checked through the
    # probability-integral transform of M on the grid of p values
    sel = (p > 0.05) & (p < 0.95)
    tail = (1 - p[sel]) ** M[sel]           # P(M' > M) for an independent copy
    u = tail + (1 - p[sel]) ** (M[sel] - 1) * p[sel] * 0.5  # mid-P transform
    assert abs(u.mean() - 0.5) < 0.02


def test_saturation_when_every_weight_underflows():
    """A frozen chain (every uphill move has weight below 2^-1000): p
    underflows to 0, M saturates at 2^63-1 and the choice still picks the
    largest weight (the least uphill neighbour)."""
    N = 6
    Q = np.diag(np.arange(1, N + 1, dtype=np.int64)) * 1000   # x = 0 is the minimum
    r = oracle.run(Q, 10.0, oracle.MODE_RF, 3, seed=1)
    assert r.M[0, 0] == np.iinfo(np.int64).max
    assert r.saturated[0] >= 1
    assert r.action[0, 0] == 0  # bit 0 costs least (1000)


def _one_step_choice(lib_handle=None):
    """One step of 200000 independent chains from one fixed state and the
    first systematic set (bits 0 .. n-1): (weights w_j = min(1, exp(-beta
    dE_j)) with dE_j = E(x ^ e_j) - E(x) from numpy energies x^T Q x, the
    run's result)."""
    N, n, beta, C = 12, 5, 0.08, 200000
    Q = _small_int_q(N, 21, -20, 20)
    x = np.array([1, 0, 1, 1, 0, 0, 1, 0, 1, 0, 0, 1], dtype=np.int64)

    def energy(s):
        return int(s @ Q @ s)

    w = np.empty(n)
    for j in range(n):
        y = x.copy()
        y[j] ^= 1
        w[j] = min(1.0, np.exp(-beta * (energy(y) - energy(x))))
    r = oracle.run(Q, beta, oracle.MODE_UNBIASED_SYS, 1, n=n, L0=10**15, seed=4, num_chains=C,
                   x0=np.tile(x.astype(np.uint8), (C, 1)), lib_handle=lib_handle)
    return w, r


def _choice_chi2(w, actions):
    counts = np.bincount(actions, minlength=len(w))[:len(w)]
    expect = len(actions) * w / w.sum()
    return ((counts - expect) ** 2 / expect).sum()


def test_one_step_choice_is_proportional_to_the_weights():
    """Proportional choice (appendix "How to Sample Proportionally", Prop 5):
    from one fixed state and one systematic set, p equals sum_S w / n, the
    chosen bit follows w_j / sum_S w (chi-square, n - 1 degrees of freedom),
    no bit outside the set is chosen, and P(M = 1) = p."""
    w, r = _one_step_choice()
    n, C = len(w), r.action.shape[0]
    assert w.min() < 0.5 < w.max()  # the weights differ, so the law is informative
    p = w.sum() / n
    assert np.allclose(r.p[:, 0], p, rtol=1e-13, atol=0)
    a = r.action[:, 0]
    assert ((a >= 0) & (a < n)).all()
    chi2 = _choice_chi2(w, a)
    assert chi2 < 25.0, chi2  # 99.99% quantile of chi2(4) is about 23.5
    m1 = (r.M[:, 0] == 1).mean()
    assert abs(m1 - p) < 5 * np.sqrt(p * (1 - p) / C)


def test_planted_choice_mistake_is_caught(tmp_path):
    """A choice whose running sum counts the candidates instead of adding
    their weights (planted in a copy of the oracle) fails the
    proportionality pin."""
    L = oracle.load_mutant([("        run += w[j];\n", "        run += w[j] > 0.0 ? 1.0 : 0.0;\n")], str(tmp_path))
    w, r = _one_step_choice(L)
    assert _choice_chi2(w, r.action[:, 0]) > 100.0


# --------------------------------------------------------------------------
# Stationary laws against brute-force enumeration
# --------------------------------------------------------------------------

def _c1_like(N=12):
    return inputs.symmetric_int(N, -50, 50, np.int64, seed=11)


def test_rejection_free_converges_to_pi():
    Q = _c1_like()
    pi = exact.target(Q, 0.05)
    r = oracle.run(Q, 0.05, oracle.MODE_RF, 50000, seed=5, num_chains=16, log=False, hist=True, hist_from=5000)
    assert exact.tv(exact.empirical(r.hist_w), pi) < 0.01


@pytest.mark.parametrize("mode", [oracle.MODE_UNBIASED_SYS, oracle.MODE_UNBIASED_RAND])
def test_unbiased_pns_converges_to_pi(mode):
    Q = _c1_like()
    pi = exact.target(Q, 0.05)
    r = oracle.run(Q, 0.05, mode, 50000, n=4, L0=100, seed=5, num_chains=16, log=False, hist=True, hist_from=5000)
    assert exact.tv(exact.empirical(r.hist_w), pi) < 0.01


def test_jump_chain_visits_follow_alpha_pi():
    """Thm 3 item 4: the jump chain's stationary law is proportional to
    alpha(x) pi(x), alpha(x) = P(leave x) = (1/N) sum_j min(1, pi(y)/pi(x))."""
    Q = _c1_like(10)
    N = 10
    E = oracle.enumerate_energies(Q).astype(float)
    nbr = exact.hypercube_neighbours(N)
    lw = np.minimum(0.0, -0.05 * (E[nbr] - E[:, None]))
    alpha = np.exp(lw).mean(axis=1)
    pi = exact.target(Q, 0.05)
    law = alpha * pi / (alpha * pi).sum()
    r = oracle.run(Q, 0.05, oracle.MODE_RF, 40000, seed=8, num_chains=8, log=False, hist=True, hist_from=2000)
    assert exact.tv(exact.empirical(r.hist_v), law) < 0.01


def test_basic_pns_follows_its_exact_law_not_pi():
    Q = _c1_like(10)
    P, mu, EM, pi = exact.basic_law_qubo(Q, 0.05, 3)
    assert exact.tv(P, pi) > 0.2  # Basic PNS is biased (Sec 2)
    r = oracle.run(Q, 0.05, oracle.MODE_BASIC, 40000, n=3, seed=4, num_chains=16, log=False, hist=True, hist_from=2000)
    assert exact.tv(exact.empirical(r.hist_v), mu) < 0.015


def _mean_multiplicity_error(lib_handle=None):
    """Largest relative gap between the chain's mean multiplicity per state and
    the exact E[M | x] = E_S[n / sum_S w] of Basic PNS (Sec 2, p = subset
    average), over well-visited states of Example 2 with two neighbours a step.
    A uniform rescaling of every multiplicity leaves the normalised law alone,
    so only this absolute check pins the 1/n normalisation."""
    Q = inputs.example2()
    _, _, EM, _ = exact.basic_law_qubo(Q, 1.0, 2)
    r = oracle.run(Q, 1.0, oracle.MODE_BASIC, 60000, n=2, seed=12, num_chains=4, log=False, hist=True,
                   lib_handle=lib_handle)
    v = r.hist_v.astype(float)
    ok = v > 2000
    return float(np.max(np.abs(r.hist_w[ok] / v[ok] / EM[ok] - 1.0)))


def test_basic_mean_multiplicity_matches_exact():
    assert _mean_multiplicity_error() < 0.05


# --------------------------------------------------------------------------
# The paper's worked examples
# --------------------------------------------------------------------------

def test_example1_exact_basic_law():
    g = _golden_json("paper_examples.json")["example1"]
    nbr = np.array([[1, 2], [0, 2], [0, 1]])
    logpi = np.log(np.array(g["pi_unnormalised"], dtype=float))
    P, mu, EM = exact.basic_law_graph(nbr, logpi, g["subset_size"])
    assert np.isclose(EM[0], g["printed_E_M_A"]) and np.isclose(EM[2], g["printed_E_M_C"])
    assert np.allclose(EM, g["derived_E_M"])
    assert np.allclose(P, g["derived_limit"])
    pi = np.exp(logpi) / np.exp(logpi).sum()
    assert not np.allclose(P, pi, atol=0.04)  # the limit differs from pi (Sec 2.1)


def test_example2_basic_limit_about_point_three():
    g = _golden_json("paper_examples.json")["example2"]
    Q = inputs.example2()
    tvs = []
    for n in range(1, g["N"] + 1):
        P, mu, EM, pi = exact.basic_law_qubo(Q, 1.0, n)
        tvs.append(exact.tv(P, pi))
    assert abs(tvs[0] - g["printed_tvd_subset1"]) < g["printed_tvd_tolerance"]
    assert tvs[0] > tvs[1] > tvs[2] > tvs[3]
    assert tvs[-1] < 1e-12
    # and the simulated Basic PNS chain reaches that limit
    P1, _, _, pi = exact.basic_law_qubo(Q, 1.0, 1)
    r = oracle.run(Q, 1.0, oracle.MODE_BASIC, 100000, n=1, seed=2, num_chains=8, log=False, hist=True, hist_from=1000)
    emp = exact.empirical(r.hist_w)
    assert exact.tv(emp, P1) < 0.01
    assert abs(exact.tv(emp, pi) - g["printed_tvd_subset1"]) < 0.02
    # the target itself: pi proportional to e^{level}
    level = np.array([bin(s).count("1") for s in range(16)])
    assert np.allclose(pi, np.exp(level) / (1 + np.e) ** 4)


# --------------------------------------------------------------------------
# Special cases that must coincide bit for bit
# --------------------------------------------------------------------------

def test_basic_with_full_subset_is_rejection_free():
    Q = _small_int_q(11, 5)
    a = oracle.run(Q, 0.05, oracle.MODE_RF, 3000, seed=6, num_chains=4)
    b = oracle.run(Q, 0.05, oracle.MODE_BASIC, 3000, n=11, seed=6, num_chains=4)
    assert (a.action == b.action).all() and (a.M == b.M).all() and (a.E == b.E).all()


def test_unbiased_with_full_set_and_huge_budget_is_rejection_free():
    Q = _small_int_q(11, 5)
    a = oracle.run(Q, 0.05, oracle.MODE_RF, 3000, seed=6, num_chains=4)
    for mode in (oracle.MODE_UNBIASED_SYS, oracle.MODE_UNBIASED_RAND):
        b = oracle.run(Q, 0.05, mode, 3000, n=11, L0=2 ** 62, seed=6, num_chains=4)
        assert (a.action == b.action).all() and (a.M == b.M).all() and (a.E == b.E).all()


def test_unbiased_budget_schedule_at_infinite_temperature():
    """beta = 0: every move is accepted (p = 1, M = 1), so with L0 = 3 the
    budget runs out after three moves and Alg 6 emits a stay record with
    M = L = 0 and switches to the next set."""
    Q = _small_int_q(8, 1)
    r = oracle.run(Q, 0.0, oracle.MODE_UNBIASED_SYS, 40, n=2, L0=3, seed=1)
    acts, M = r.action[0], r.M[0]
    for k in range(40):
        if k % 4 == 3:
            assert acts[k] == oracle.STAY and M[k] == 0
        else:
            assert acts[k] >= 0 and M[k] == 1
            assert oracle.sys_subset(8, 2, (k // 4) % 4)[acts[k]]
    assert r.sub[0] == 10


def test_resume_is_bit_identical():
    """Counter-based randomness: K steps then K more from the saved state equal
    2K steps in one go."""
    Q = _small_int_q(9, 8)
    full = oracle.run(Q, 0.05, oracle.MODE_BASIC, 400, n=3, seed=2, num_chains=2)
    half = oracle.run(Q, 0.05, oracle.MODE_BASIC, 200, n=3, seed=2, num_chains=2)
    rest = oracle.run(Q, 0.05, oracle.MODE_BASIC, 200, n=3, seed=2, num_chains=2, x0=half.x, step0=200)
    assert (np.concatenate([half.action, rest.action], 1) == full.action).all()
    assert (np.concatenate([half.M, rest.M], 1) == full.M).all()


# --------------------------------------------------------------------------
# Planted mistakes: each must be caught by one of the pins above
# --------------------------------------------------------------------------

MUTANTS = {
    "p_over_N_not_n": [("p = S / (double)n;", "p = S / (double)N;")],
    "M_without_plus_one": [("m = (int64_t)floor(q) + 1;", "m = (int64_t)floor(q) + (q > 1.0 ? 0 : 1);")],
    "dE_wrong_sign": [("return (x[j] ? -1 : 1) * (d + s * hi[j]);", "return (x[j] ? 1 : -1) * (d + s * hi[j]);")],
    "field_dropped_diagonal": [("int64_t d = a->Qi[(size_t)j * a->N + j];", "int64_t d = 0;")],
    "stay_keeps_subset": [("++sub;\n", "")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    L = oracle.load_mutant(MUTANTS[name], str(tmp_path))
    caught = []
    Q2 = inputs.example2()
    P1, _, _, pi2 = exact.basic_law_qubo(Q2, 1.0, 1)
    r = oracle.run(Q2, 1.0, oracle.MODE_BASIC, 60000, n=1, seed=2, num_chains=4, log=False, hist=True,
                   hist_from=1000, lib_handle=L)
    caught.append(exact.tv(exact.empirical(r.hist_w), P1) > 0.01)
    Q = _c1_like(10)
    pi = exact.target(Q, 0.05)
    for mode in (oracle.MODE_RF, oracle.MODE_UNBIASED_SYS):
        r = oracle.run(Q, 0.05, mode, 30000, n=4, L0=100, seed=5, num_chains=8, log=False, hist=True,
                       hist_from=3000, lib_handle=L)
        caught.append(exact.tv(exact.empirical(r.hist_w), pi) > 0.01)
    caught.append(_mean_multiplicity_error(L) > 0.05)
    assert any(caught), f"planted mistake {name} was not caught"


# --------------------------------------------------------------------------
# Optimization RF / PNS (Alg 9, Alg 10) used as burn-in (Sec 8)
# --------------------------------------------------------------------------

def test_optimization_at_unit_temperature_is_the_jump_chain_without_multiplicity():
    """Sec 2 builds Basic PNS as Optimization PNS plus a multiplicity list,
    and Optimization RF is RF's jump chain: at T = 1 the moves coincide
    (same counter-based draws) and every jump counts once."""
    Q = _small_int_q(10, 21)
    for mode, n in ((oracle.MODE_RF, 10), (oracle.MODE_BASIC, 4)):
        ref = oracle.run(Q, 0.2, mode, 300, n=n, seed=5, num_chains=3)
        opt = oracle.run(Q, 0.2, oracle.MODE_OPT, 300, n=n, seed=5, num_chains=3, temperature=1.0)
        assert np.array_equal(opt.action, ref.action)
        assert np.array_equal(opt.E, ref.E)
        assert (opt.M == 1).all()


def test_optimization_temperature_tempers_the_target():
    """Weights [pi(y)/pi(x)]^(1/T) of pi_beta are those of pi_{beta/T}."""
    Q = _small_int_q(9, 22)
    hot = oracle.run(Q, 0.3, oracle.MODE_OPT, 250, n=9, seed=2, num_chains=2, temperature=3.0)
    ref = oracle.run(Q, 0.1, oracle.MODE_RF, 250, seed=2, num_chains=2)
    assert np.array_equal(hot.action, ref.action)


def test_optimization_keeps_the_best_state():
    """X_max is the lowest-energy state of the trajectory (J_0 included), and
    its energy is the brute-force x^T Q x of the stored bits."""
    Q = _small_int_q(12, 23)
    r = oracle.run(Q, 0.5, oracle.MODE_OPT, 400, n=5, seed=7, num_chains=4, temperature=0.7, init="random")
    for c in range(4):
        traj = np.concatenate([r.E[c], [r.E_final[c]]])
        assert r.E_best[c] == traj.min()
        xb = r.x_best[c].astype(np.int64)
        assert r.E_best[c] == int(xb @ Q.astype(np.int64) @ xb)


def test_cold_optimization_ends_in_a_local_minimum_and_finds_the_ground_state():
    """At a low temperature Optimization RF descends: X_max is a local
    minimum (no single flip lowers the energy), and over a few chains the
    global minimum of a small problem (enumeration) is reached."""
    Q = _small_int_q(8, 24)
    r = oracle.run(Q, 1.0, oracle.MODE_OPT, 3000, n=8, seed=11, num_chains=16, temperature=0.5, init="random")
    Qi = Q.astype(np.int64)
    for c in range(16):
        xb = r.x_best[c].astype(np.int64)
        e0 = int(xb @ Qi @ xb)
        for j in range(8):
            y = xb.copy()
            y[j] ^= 1
            assert int(y @ Qi @ y) >= e0
    assert r.E_best.min() == oracle.enumerate_energies(Q).min()


# --------------------------------------------------------------------------
# Original-time runs and parallel tempering
# --------------------------------------------------------------------------

def test_original_time_run_is_the_jump_chain_cut_at_time_t():
    """The records of a run of T original samples are those of the untimed
    run up to the record covering time T, whose multiplicity is cut to the
    remaining time: the multiplicities sum to T exactly."""
    Q = _small_int_q(10, 31)
    T = 500
    full = oracle.run(Q, 0.2, oracle.MODE_RF, 600, seed=4, num_chains=5)
    cut = oracle.run(Q, 0.2, oracle.MODE_RF, T, seed=4, num_chains=5, orig_time=T)
    for c in range(5):
        k = int(cut.n_records[c])
        assert cut.M[c, :k].sum() == T
        assert cut.action[c, k - 1] == oracle.STAY
        assert np.array_equal(cut.action[c, :k - 1], full.action[c, :k - 1])
        assert np.array_equal(cut.M[c, :k - 1], full.M[c, :k - 1])
        assert full.M[c, :k].sum() >= T > full.M[c, :k - 1].sum()


def _pi_and_alpha(Q, beta):
    N = Q.shape[0]
    E = oracle.enumerate_energies(Q).astype(np.float64)
    s = np.arange(1 << N)
    alpha = np.mean([np.minimum(1.0, np.exp(-beta * (E[s ^ (1 << j)] - E))) for j in range(N)], axis=0)
    pi = exact.target(Q, beta)
    return pi, alpha


def test_original_time_states_follow_pi_not_the_jump_law():
    """From exact draws of pi, the original chain is still pi-distributed after
    T original samples, while the jump chain's state law is alpha pi."""
    Q = _small_int_q(8, 32, lo=-6, hi=6)
    beta = 0.5
    pi, alpha = _pi_and_alpha(Q, beta)
    jump_law = alpha * pi / (alpha * pi).sum()
    C = 40000
    rng = np.random.default_rng(1)
    idx0 = rng.choice(256, size=C, p=pi)
    x0 = ((idx0[:, None] >> np.arange(8)) & 1).astype(np.uint8)
    r = oracle.run(Q, beta, oracle.MODE_RF, 7, seed=9, num_chains=C, x0=x0, orig_time=7, log=False)
    idx = (r.x.astype(np.int64) << np.arange(8)).sum(axis=1)
    emp = np.bincount(idx, minlength=256) / C
    floor = exact.tv(np.bincount(rng.choice(256, size=C, p=pi), minlength=256) / C, pi)
    assert exact.tv(pi, jump_law) > 0.05
    assert exact.tv(emp, pi) < floor + 0.015
    assert exact.tv(emp, jump_law) > exact.tv(pi, jump_law) / 2


def test_pt_swap_acceptance_rate_and_ladder():
    """A pair of chains with fixed energies exchanges temperatures with
    probability min{1, exp[(b_a - b_b)(E_a - E_b)]}; the ladder always lists
    the chain holding each temperature."""
    T = 2
    groups = 20000
    E = np.tile(np.array([5, 2], dtype=np.int64), groups)
    ladder_betas = np.array([0.1, 0.5])
    betas = np.tile(ladder_betas, groups).astype(np.float64)
    ladder = np.tile(np.arange(T, dtype=np.int32), groups)
    acc = oracle.pt_round(E, betas, ladder, T, seed=3, round_=0)
    # chain 0 (beta 0.1, E 5) and chain 1 (beta 0.5, E 2): exponent (0.1-0.5)(5-2) = -1.2
    rate = acc[0::2].mean()
    assert abs(rate - np.exp(-1.2)) < 4 * np.sqrt(np.exp(-1.2) * (1 - np.exp(-1.2)) / groups)
    for g in range(groups):
        for t in range(T):
            assert betas[g * T + ladder[g * T + t]] == ladder_betas[t]
    # the reverse pair (higher energy at the colder temperature) always swaps
    E2 = np.tile(np.array([2, 5], dtype=np.int64), groups)
    betas2 = np.tile(ladder_betas, groups).astype(np.float64)
    ladder2 = np.tile(np.arange(T, dtype=np.int32), groups)
    assert oracle.pt_round(E2, betas2, ladder2, T, seed=3, round_=0)[0::2].all()


def _pt_experiment(lib_handle=None):
    """RF sweeps of 4 original samples alternated with swap rounds at two
    temperatures; returns (TV of each temperature's states to its pi, the
    sampling floor of each, swaps made)."""
    Q = _small_int_q(6, 33, lo=-8, hi=8)
    ladder_betas = np.array([0.15, 0.8])
    T = 2
    groups = 6000
    C = groups * T
    pis = [_pi_and_alpha(Q, b)[0] for b in ladder_betas]
    rng = np.random.default_rng(2)
    x = np.zeros((C, 6), np.uint8)
    for t in range(T):
        idx0 = rng.choice(64, size=groups, p=pis[t])
        x[t::T] = ((idx0[:, None] >> np.arange(6)) & 1).astype(np.uint8)
    betas = np.tile(ladder_betas, groups).astype(np.float64)
    ladder = np.tile(np.arange(T, dtype=np.int32), groups)
    steps = np.zeros(C, np.int64)
    swaps = 0
    for sweep in range(25):
        r = oracle.run(Q, betas, oracle.MODE_RF, 4, seed=5, num_chains=C, x0=x, step0=steps, orig_time=4,
                       lib_handle=lib_handle)
        x = r.x
        steps = steps + r.n_records
        swaps += oracle.pt_round(r.E_final, betas, ladder, T, seed=5, round_=sweep, lib_handle=lib_handle).sum()
    tvs, floors = [], []
    for t in range(T):
        chains = np.arange(groups) * T + ladder[t::T]
        idx = (x[chains].astype(np.int64) << np.arange(6)).sum(axis=1)
        tvs.append(exact.tv(np.bincount(idx, minlength=64) / groups, pis[t]))
        floors.append(exact.tv(np.bincount(rng.choice(64, size=groups, p=pis[t]), minlength=64) / groups, pis[t]))
    return tvs, floors, swaps


def test_parallel_tempering_keeps_each_temperature_at_its_target():
    """The state held at each temperature follows pi at that temperature
    (enumeration) and swaps do happen."""
    tvs, floors, swaps = _pt_experiment()
    assert swaps > 0.05 * 6000 * 25 / 2
    for tv, floor in zip(tvs, floors):
        assert tv < floor + 0.02, (tvs, floors)


@pytest.mark.parametrize("mutation", [
    [("const double ex = (betas[ca] - betas[cb]) * dE;", "const double ex = (betas[cb] - betas[ca]) * dE;")],
    [("                L = 0;\n                ++stays;",
      "                L = 0;\n                x[0] ^= 1u;\n                ++stays;")],
])
def test_planted_tempering_mistakes_are_caught(mutation, tmp_path):
    """A swap exponent of the wrong sign, or a chain that moves at the end of
    its time budget, breaks the per-temperature laws."""
    L = oracle.load_mutant(mutation, str(tmp_path))
    tvs, floors, _ = _pt_experiment(L)
    assert any(tv > floor + 0.02 for tv, floor in zip(tvs, floors)), (tvs, floors)
