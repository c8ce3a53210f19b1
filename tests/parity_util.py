"""Helpers shared by the GPU parity tests: run the HIP sampler and the CPU
oracle on the same seeded input and compare their records element by element.

Integer Q: actions, multiplicities, energies and local fields must be equal
bit for bit.  A differing action or multiplicity is tolerated only where the
oracle shows the step sat on an FP64 decision boundary (its quotient q within
1e-9 relative of the integer or budget it is compared with, or U2*S within
1e-9 of a cumulative-sum boundary); the comparison of that chain then stops
there.  No such case is expected at these sizes.  Float Q: the same, with
energies and fields to a relative 1e-9 of the FP64 oracle (the declared
tolerance is 1e-5)."""
from __future__ import annotations

import numpy as np

import oracle

MODE_IDS = {"rf": oracle.MODE_RF, "basic": oracle.MODE_BASIC, "unbiased_sys": oracle.MODE_UNBIASED_SYS,
            "unbiased_rand": oracle.MODE_UNBIASED_RAND}


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


def oracle_run(Q, beta, mode, K, *, n=0, L0=100, seed=0, chains=None, init="zero", layout="symmetric", x0=None):
    lay = oracle.LAYOUT_UPPER if layout == "upper" else oracle.LAYOUT_SYMMETRIC
    cids = np.asarray(chains, dtype=np.uint32)
    Qo = Q.astype(np.int64) if np.issubdtype(Q.dtype, np.integer) else Q.astype(np.float64)
    return oracle.run(Qo, beta, MODE_IDS[mode], K, n=n, L0=L0, seed=seed, num_chains=len(cids), chain_ids=cids,
                      init=init, layout=lay, x0=x0)


def _boundary(o, c, k, L_before=None):
    q = o.q[c, k]
    if np.isfinite(q) and q > 0:
        frac = abs(q - np.round(q)) / max(1.0, q)
        if frac < 1e-9:
            return True
    return o.tmargin[c, k] < 1e-9


def compare_logs(g, o, *, chain_rows, is_int, rtol=1e-9, p_rtol=1e-12):
    """g: gpu log dict restricted to chain_rows; o: oracle result of the same
    chains in the same order.  Returns the number of steps compared."""
    ga, gM, gE, gp = (g["action"][chain_rows], g["M"][chain_rows], g["E"][chain_rows], g["p"][chain_rows])
    compared = 0
    for c in range(len(chain_rows)):
        same = (ga[c] == o.action[c]) & (gM[c] == o.M[c])
        bad = np.nonzero(~same)[0]
        upto = len(same) if len(bad) == 0 else bad[0]
        if len(bad):
            k = bad[0]
            assert _boundary(o, c, k), (
                f"chain row {c}: step {k} differs off any FP boundary: gpu (a={ga[c, k]}, M={gM[c, k]}) "
                f"oracle (a={o.action[c, k]}, M={o.M[c, k]}, q={o.q[c, k]!r}, tmargin={o.tmargin[c, k]!r})")
        if is_int:
            assert np.array_equal(gE[c, :upto], o.E[c, :upto].astype(np.float64)), f"chain row {c}: energies differ"
        else:
            assert np.allclose(gE[c, :upto], o.E[c, :upto], rtol=rtol, atol=rtol), f"chain row {c}: energies differ"
        okp = np.isclose(gp[c, :upto], o.p[c, :upto], rtol=p_rtol, atol=0)
        if not okp.all():
            k = int(np.nonzero(~okp)[0][0])
            raise AssertionError(f"chain row {c}: p differs at step {k}: gpu {gp[c, k]!r} oracle {o.p[c, k]!r}")
        compared += upto
    return compared


def compare_final(gcur, o, *, chain_rows, is_int, rtol=1e-9):
    gx, gh, gE = gcur["x"][chain_rows], gcur["h"][chain_rows], gcur["E"][chain_rows]
    assert np.array_equal(gx, o.x), "final states differ"
    if is_int:
        assert np.array_equal(gh.astype(np.int64), o.h), "final fields differ"
        assert np.array_equal(gE, o.E_final.astype(np.float64)), "final energies differ"
    else:
        scale = np.maximum(1.0, np.abs(o.h).max())
        assert np.max(np.abs(gh - o.h)) <= rtol * scale, "final fields differ"
        assert np.allclose(gE, o.E_final, rtol=rtol, atol=rtol), "final energies differ"
