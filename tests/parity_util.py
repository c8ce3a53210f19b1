"""Helpers shared by the GPU parity tests: run the HIP sampler and compare its
records with the CPU oracle element by element, through the oracle's replay
mode.

Replay feeds the GPU's records (action, M) of each chain to the oracle, which
derives from its own state and its own Philox draws the energy, the weights,
p, q and its own decision at every record, classifies the GPU's decision, and
continues along the GPU's trajectory.  So every record of every compared
chain is checked, and the final state is always compared:
  - integer Q: energies and local fields equal bit for bit; float Q: to a
    relative 1e-9 of the FP64 oracle (the declared tolerance is 1e-5);
  - p to a relative P_RTOL (the two sides sum the same weights in different
    orders; integer Q weights come from tables on the GPU, a few ulp apart);
  - the decision (chosen bit, multiplicity, stay) equal, except where the
    oracle shows that it sits on a decision boundary: q within the band
    that a relative P_RTOL in p can move it across of the budget L or of the
    interval [M - 1, M) of the GPU's multiplicity, or U2*S within 2 P_RTOL S
    of an end of the GPU's chosen interval.  Such records are counted
    ("exempt") and still compared in everything else.  Their number must stay
    within what the windows allow (max_exempt): about zero for ordinary
    records, up to one per record where q is so large (p below ~1e-12, nearly
    frozen chains) that the window spans integers.  A decision off every
    window fails the test.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle

MODE_IDS = {"rf": oracle.MODE_RF, "basic": oracle.MODE_BASIC, "unbiased_sys": oracle.MODE_UNBIASED_SYS,
            "unbiased_rand": oracle.MODE_UNBIASED_RAND, "opt": oracle.MODE_OPT}

P_RTOL = 1e-12   # p of the two sides (summation order, table exponentials)
E_RTOL = 1e-9    # float-Q energies and fields against the FP64 oracle


@dataclass
class Coverage:
    compared: int = 0          # records compared (decision classified, E and p checked)
    exempt: int = 0            # of which decision-boundary cases (still compared)
    finals: int = 0            # chains whose final state was compared
    classes: dict = field(default_factory=dict)

    def add(self, other: "Coverage") -> None:
        self.compared += other.compared
        self.exempt += other.exempt
        self.finals += other.finals
        for k, v in other.classes.items():
            self.classes[k] = self.classes.get(k, 0) + v


SESSION = Coverage()   # totals over the test session (printed by conftest)


def window_width(p, q, tol):
    """Half-width, in units of q, of the band around a boundary of
    q = log U1 / log1p(-p) that a relative difference `tol` in p can move q
    across: kappa(p) tol q + 8 ulp, kappa(p) = p / ((1 - p) |log1p(-p)|)."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = np.where((p > 0) & (p < 1), p / ((1 - p) * np.abs(np.log1p(-p))),
                         1.0)
    kappa = np.where(np.isfinite(kappa), kappa, 1.0)
    w = (kappa * tol + 8 * 2.0 ** -52) * np.where(np.isfinite(q), np.abs(q), 0.0)
    return np.where(np.isfinite(q), w, np.inf)


def max_exempt(p, q, tol) -> float:
    """Boundary cases allowed among records with these p and q: the expected
    number of records whose q-window holds a boundary if q fell anywhere
    (sum of min(1, 2 w)), plus two for the choice windows.  Records with
    q beyond about 1 / tol (nearly frozen chains, p ~ 1e-20 and below) have
    windows wider than one integer: their multiplicity differs between any
    two computations of p and is only checked to lie inside its window."""
    return 2.0 + float(np.minimum(1.0, 2.0 * window_width(p, q, tol)).sum())


def gpu_run(Q, beta, mode, K, *, n=0, L0=100, seed=0, chains=1, init="zero", layout="symmetric",
            launch="persistent", chunk=0, block=0, groups=0, chain_id_base=0, log=True, x0=None):
    from paper_2210_10513_amd.binding import Sampler
    s = Sampler(Q, beta, n, mode, num_chains=chains, L0=L0, seed=seed, init=init, x0=x0, layout=layout,
                launch=launch, chunk=chunk, block=block, groups=groups, log_capacity=K if log else 0,
                chain_id_base=chain_id_base)
    s.run(K)
    from paper_2210_10513_amd.binding import pns_problem_info_get
    out = {"log": s.read_log() if log else None, "cur": s.read_current(), "rec": s.read(), "stats": s.stats(),
           "tile": s.tile(), "flavour": pns_problem_info_get(s.ctx, 0).flavour}
    s.close()
    return out


def _oracle_q(Q):
    return Q.astype(np.int64) if np.issubdtype(Q.dtype, np.integer) else Q.astype(np.float64)


def _layout(layout):
    return oracle.LAYOUT_UPPER if layout == "upper" else oracle.LAYOUT_SYMMETRIC


def oracle_run(Q, beta, mode, K, *, n=0, L0=100, seed=0, chains=None, init="zero", layout="symmetric", x0=None,
               **kw):
    cids = np.asarray(chains, dtype=np.uint32)
    return oracle.run(_oracle_q(Q), beta, MODE_IDS.get(mode, mode), K, n=n, L0=L0, seed=seed, num_chains=len(cids),
                      chain_ids=cids, init=init, layout=_layout(layout), x0=x0, **kw)


def _describe(o, glog_rows, c, k):
    return (f"chain row {c}, record {k}: gpu (action={glog_rows['action'][c, k]}, M={glog_rows['M'][c, k]}) "
            f"oracle (action={o.action[c, k]}, M={o.M[c, k]}, q={o.q[c, k]!r}, p={o.p[c, k]!r}, "
            f"class={oracle.RP_NAMES.get(int(o.cls[c, k]))})")


def replay_check(glog, Q, beta, mode, *, rows, chain_ids=None, is_int, lengths=None, p_rtol=P_RTOL, rtol=E_RTOL,
                 gcur=None, n=0, L0=100, seed=0, init="zero", layout="symmetric", x0=None, step0=0,
                 temperature=1.0, orig_time=0):
    """Replay the GPU log rows `rows` (chain ids `chain_ids`, default = rows)
    through the oracle and compare every record; with `gcur` also the final
    states, fields and energies.  `lengths` (per row) limits the records
    compared (exact-time runs stop early).  Returns (oracle result, Coverage)."""
    rows = list(rows)
    cids = np.asarray(rows if chain_ids is None else chain_ids, dtype=np.uint32)
    g = {k: np.ascontiguousarray(v[rows]) for k, v in glog.items()}
    K = g["action"].shape[1]
    betas = np.broadcast_to(np.asarray(beta, dtype=np.float64), (len(rows),))
    o = oracle.replay(_oracle_q(Q), betas, MODE_IDS.get(mode, mode), g["action"], g["M"], tol=p_rtol, n=n, L0=L0,
                      seed=seed, num_chains=len(rows), chain_ids=cids, init=init, layout=_layout(layout), x0=x0,
                      step0=step0, temperature=temperature, orig_time=orig_time)
    cov = Coverage()
    lens = np.full(len(rows), K) if lengths is None else np.asarray(lengths)
    allowed = 0.0
    for c in range(len(rows)):
        m = int(lens[c])
        cls = o.cls[c, :m]
        bad = np.nonzero(cls < 0)[0]
        assert len(bad) == 0, "decision off every boundary window: " + _describe(o, g, c, int(bad[0]))
        if is_int:
            diff = np.nonzero(g["E"][c, :m] != o.E[c, :m].astype(np.float64))[0]
        else:
            diff = np.nonzero(~np.isclose(g["E"][c, :m], o.E[c, :m], rtol=rtol, atol=rtol))[0]
        assert len(diff) == 0, f"chain row {c}: energy differs at record {diff[0]}: gpu {g['E'][c, diff[0]]!r} " \
                               f"oracle {o.E[c, diff[0]]!r}"
        okp = np.isclose(g["p"][c, :m], o.p[c, :m], rtol=p_rtol, atol=0)
        if not okp.all():
            k = int(np.nonzero(~okp)[0][0])
            raise AssertionError(f"chain row {c}: p differs at record {k}: gpu {g['p'][c, k]!r} oracle {o.p[c, k]!r}")
        cov.compared += m
        cov.exempt += int((cls > 0).sum())
        allowed += max_exempt(o.p[c, :m], o.q[c, :m], p_rtol)
        for v, cnt in zip(*np.unique(cls, return_counts=True)):
            cov.classes[oracle.RP_NAMES[int(v)]] = cov.classes.get(oracle.RP_NAMES[int(v)], 0) + int(cnt)
    if gcur is not None:
        compare_final(gcur, o, chain_rows=rows, is_int=is_int, rtol=rtol)
        cov.finals += len(rows)
    assert cov.exempt <= allowed, f"more decision-boundary cases than their windows allow ({allowed:.1f}): {cov}"
    SESSION.add(cov)
    return o, cov


def compare_final(gcur, o, *, chain_rows, is_int, rtol=E_RTOL):
    gx, gh, gE = gcur["x"][chain_rows], gcur["h"][chain_rows], gcur["E"][chain_rows]
    assert np.array_equal(gx, o.x), "final states differ"
    if is_int:
        assert np.array_equal(gh.astype(np.int64), o.h), "final fields differ"
        assert np.array_equal(gE, o.E_final.astype(np.float64)), "final energies differ"
    else:
        scale = np.maximum(1.0, np.abs(o.h).max())
        assert np.max(np.abs(gh - o.h)) <= rtol * scale, "final fields differ"
        assert np.allclose(gE, o.E_final, rtol=rtol, atol=rtol), "final energies differ"


def cont_replay_check(glog, x0, *, p_rtol, rtol, chain_ids=None, **kw):
    """Continuous Unbiased PNS: replay the GPU's records through the oracle
    (``oracle.cont_run`` with ``follow``) and compare every record's log
    density and p; returns (oracle result, Coverage)."""
    C, K = glog["action"].shape
    o = oracle.cont_run(x0, K, chain_ids=chain_ids, follow=(glog["action"], glog["M"]), follow_tol=p_rtol, **kw)
    cov = Coverage()
    for c in range(C):
        bad = np.nonzero(o.cls[c] < 0)[0]
        assert len(bad) == 0, "decision off every boundary window: " + _describe(o, glog, c, int(bad[0]))
        assert np.allclose(glog["E"][c], o.E[c], rtol=rtol, atol=rtol), f"chain {c}: log densities differ"
        okp = np.isclose(glog["p"][c], o.p[c], rtol=p_rtol, atol=0)
        if not okp.all():
            k = int(np.nonzero(~okp)[0][0])
            raise AssertionError(f"chain {c}: p differs at record {k}: gpu {glog['p'][c, k]!r} oracle {o.p[c, k]!r}")
        cov.compared += K
        cov.exempt += int((o.cls[c] > 0).sum())
        for v, cnt in zip(*np.unique(o.cls[c], return_counts=True)):
            cov.classes[oracle.RP_NAMES[int(v)]] = cov.classes.get(oracle.RP_NAMES[int(v)], 0) + int(cnt)
    allowed = max_exempt(o.p, o.q, p_rtol)
    assert cov.exempt <= allowed, f"more decision-boundary cases than their windows allow ({allowed:.1f}): {cov}"
    SESSION.add(cov)
    return o, cov
