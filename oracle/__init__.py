"""Reference oracle for Partial Neighbor Search sampling (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never imports it and
shares no code with it.

``pns_oracle.c`` holds the plain single-threaded FP64/int64 chain simulation
(Rejection-Free Alg 2, Basic PNS Alg 3, Unbiased PNS Alg 6 on the QUBO target
of Sec 4) and its own Philox4x32-10; this module loads it with ctypes and
``exact.py`` holds the enumeration-based exact laws used as pins;
``donut.py`` the exact moments of the continuous (donut) target by quadrature.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pns_oracle.c")
_LIB = os.path.join(_HERE, "_pns_oracle.so")

MODE_RF = 0
MODE_BASIC = 1
MODE_UNBIASED_SYS = 2
MODE_UNBIASED_RAND = 3
MODE_OPT = 4
LAYOUT_SYMMETRIC = 0
LAYOUT_UPPER = 1
STAY = -1

# Replay classes (orc_replay_class): how a followed record relates to the
# oracle's own decision at the same state and draws.
RP_SAME = 0        # same action and multiplicity
RP_BUDGET = 1      # stay vs move differs, q within the window of the budget L
RP_MULT = 2        # multiplicity differs, q within the window of the interval [M-1, M) the given M needs
RP_CHOICE = 3      # chosen neighbour differs, U2*S within the window of its interval
RP_MISMATCH = -1   # differs off every decision window
RP_INVALID = -2    # the given action is impossible at that step
RP_NAMES = {RP_SAME: "same", RP_BUDGET: "budget boundary", RP_MULT: "multiplicity boundary",
            RP_CHOICE: "choice boundary", RP_MISMATCH: "mismatch", RP_INVALID: "invalid action"}


def load_mutant(replacements, workdir: str) -> ctypes.CDLL:
    """Compile a copy of the oracle with textual replacements applied (used by
    tests that plant a mistake in the oracle to show a pin catches it)."""
    src = open(_SRC).read()
    for old, new in replacements:
        if old not in src:
            raise ValueError(f"mutation anchor not found: {old!r}")
        src = src.replace(old, new, 1)
    cpath = os.path.join(workdir, "mutant.c")
    so = os.path.join(workdir, "mutant.so")
    with open(cpath, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", so, cpath, "-lm"])
    L = ctypes.CDLL(so)
    _declare(L)
    return L


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _RunArgs(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("is_int", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("Qi", ctypes.c_void_p), ("Qf", ctypes.c_void_p),
        ("mode", ctypes.c_int32), ("n", ctypes.c_int32), ("L0", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("num_chains", ctypes.c_int32), ("chain_ids", ctypes.c_void_p), ("betas", ctypes.c_void_p),
        ("x0", ctypes.c_void_p), ("K", ctypes.c_int64), ("step0", ctypes.c_int64),
        ("log_action", ctypes.c_void_p), ("log_M", ctypes.c_void_p), ("log_Ei", ctypes.c_void_p),
        ("log_Ef", ctypes.c_void_p), ("log_p", ctypes.c_void_p), ("log_q", ctypes.c_void_p),
        ("log_tmargin", ctypes.c_void_p),
        ("x_final", ctypes.c_void_p), ("hi_final", ctypes.c_void_p), ("hf_final", ctypes.c_void_p),
        ("Ei_final", ctypes.c_void_p), ("Ef_final", ctypes.c_void_p), ("L_final", ctypes.c_void_p),
        ("sub_final", ctypes.c_void_p),
        ("hist_w", ctypes.c_void_p), ("hist_v", ctypes.c_void_p), ("hist_from", ctypes.c_int64),
        ("n_flips", ctypes.c_void_p), ("n_stays", ctypes.c_void_p), ("n_saturated", ctypes.c_void_p),
        ("temperature", ctypes.c_double), ("x_best", ctypes.c_void_p), ("Ei_best", ctypes.c_void_p),
        ("Ef_best", ctypes.c_void_p),
        ("orig_time", ctypes.c_int64), ("n_records", ctypes.c_void_p), ("step0s", ctypes.c_void_p),
        ("log_w", ctypes.c_void_p), ("hist_rb", ctypes.c_void_p),
        ("rp_action", ctypes.c_void_p), ("rp_M", ctypes.c_void_p), ("rp_class", ctypes.c_void_p),
        ("rp_tol", ctypes.c_double),
    ]


def _declare(L: ctypes.CDLL) -> None:
    u32p = ctypes.POINTER(ctypes.c_uint32)
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_philox4x32_10.restype = None
    L.orc_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.orc_uniforms.restype = None
    L.orc_random_subset.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_random_subset.restype = None
    L.orc_sys_subset.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p]
    L.orc_sys_subset.restype = None
    L.orc_sys_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.orc_sys_count.restype = ctypes.c_int64
    L.orc_random_state.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_random_state.restype = None
    L.orc_energy_i.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_energy_i.restype = ctypes.c_int64
    L.orc_energy_f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_energy_f.restype = ctypes.c_double
    L.orc_run.argtypes = [ctypes.POINTER(_RunArgs)]
    L.orc_run.restype = ctypes.c_int
    L.orc_enumerate_energies_i.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_enumerate_energies_i.restype = ctypes.c_int
    L.orc_enumerate_energies_f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_enumerate_energies_f.restype = ctypes.c_int
    L.orc_basic_onestep.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_basic_onestep.restype = ctypes.c_int
    L.orc_pt_round.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
    L.orc_pt_round.restype = ctypes.c_int
    L.orc_expected_multiplicity.argtypes = [ctypes.c_double, ctypes.c_int64]
    L.orc_expected_multiplicity.restype = ctypes.c_double
    L.orc_cont_run.argtypes = [ctypes.POINTER(_ContArgs)]
    L.orc_cont_run.restype = ctypes.c_int
    L.orc_cont_offsets.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p]
    L.orc_cont_offsets.restype = None


def _ptr(a: Optional[np.ndarray]) -> Optional[int]:
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def uniforms(seed: int, chain: int, step: int):
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_uniforms(seed, chain, step, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def random_subset(seed: int, chain: int, step: int, N: int, n: int) -> np.ndarray:
    m = np.zeros(N, dtype=np.uint8)
    lib().orc_random_subset(seed, chain, step, N, n, m.ctypes.data)
    return m.astype(bool)


def sys_subset(N: int, n: int, i: int) -> np.ndarray:
    m = np.zeros(N, dtype=np.uint8)
    lib().orc_sys_subset(N, n, i, m.ctypes.data)
    return m.astype(bool)


def sys_count(N: int, n: int) -> int:
    return int(lib().orc_sys_count(N, n))


def random_state(seed: int, chain: int, N: int) -> np.ndarray:
    x = np.zeros(N, dtype=np.uint8)
    lib().orc_random_state(seed, chain, N, x.ctypes.data)
    return x


def _as_q(Q: np.ndarray):
    Q = np.asarray(Q)
    if np.issubdtype(Q.dtype, np.integer):
        return 1, np.ascontiguousarray(Q, dtype=np.int64)
    return 0, np.ascontiguousarray(Q, dtype=np.float64)


def energy(Q: np.ndarray, x: np.ndarray, layout: int = LAYOUT_SYMMETRIC):
    is_int, Qc = _as_q(Q)
    xc = np.ascontiguousarray(x, dtype=np.uint8)
    if is_int:
        return int(lib().orc_energy_i(Qc.ctypes.data, Qc.shape[0], layout, xc.ctypes.data))
    return float(lib().orc_energy_f(Qc.ctypes.data, Qc.shape[0], layout, xc.ctypes.data))


def enumerate_energies(Q: np.ndarray, layout: int = LAYOUT_SYMMETRIC) -> np.ndarray:
    is_int, Qc = _as_q(Q)
    N = Qc.shape[0]
    if is_int:
        E = np.zeros(1 << N, dtype=np.int64)
        rc = lib().orc_enumerate_energies_i(Qc.ctypes.data, N, layout, E.ctypes.data)
    else:
        E = np.zeros(1 << N, dtype=np.float64)
        rc = lib().orc_enumerate_energies_f(Qc.ctypes.data, N, layout, E.ctypes.data)
    if rc != 0:
        raise ValueError("enumeration needs 1 <= N <= 24")
    return E


@dataclass
class RunResult:
    action: Optional[np.ndarray] = None
    M: Optional[np.ndarray] = None
    E: Optional[np.ndarray] = None      # int64 for integer Q, float64 otherwise
    p: Optional[np.ndarray] = None
    q: Optional[np.ndarray] = None
    tmargin: Optional[np.ndarray] = None
    x: Optional[np.ndarray] = None
    h: Optional[np.ndarray] = None
    E_final: Optional[np.ndarray] = None
    L: Optional[np.ndarray] = None
    sub: Optional[np.ndarray] = None
    hist_w: Optional[np.ndarray] = None
    hist_v: Optional[np.ndarray] = None
    flips: Optional[np.ndarray] = None
    stays: Optional[np.ndarray] = None
    saturated: Optional[np.ndarray] = None
    x_best: Optional[np.ndarray] = None   # MODE_OPT: best state X_max
    E_best: Optional[np.ndarray] = None
    n_records: Optional[np.ndarray] = None  # records per chain
    w: Optional[np.ndarray] = None        # expected multiplicity of each record (Rao-Blackwell weight)
    hist_rb: Optional[np.ndarray] = None  # sum of w per state
    cls: Optional[np.ndarray] = None      # replay: RP_* class of each followed record


def run(Q: np.ndarray, beta, mode: int, K: int, *, n: int = 0, L0: int = 100, seed: int = 0,
        num_chains: int = 1, chain_ids=None, x0: Optional[np.ndarray] = None, init: str = "zero",
        layout: int = LAYOUT_SYMMETRIC, log: bool = True, hist: bool = False, hist_from: int = 0,
        step0=0, lib_handle: Optional[ctypes.CDLL] = None, temperature: float = 1.0,
        orig_time: int = 0, follow=None, follow_tol: float = 0.0) -> RunResult:
    """Run ``num_chains`` independent chains for ``K`` steps each.

    ``beta`` is a scalar or one value per chain; ``init`` is ``"zero"``,
    ``"random"`` (the Bernoulli(1/2) stream) or ignored when ``x0`` is given.
    ``MODE_OPT`` runs Alg 9 (n = N) / Alg 10 (n < N) at ``temperature`` and
    fills ``x_best`` / ``E_best`` (the best state seen, X_max).  With
    ``orig_time`` > 0 (RF, Basic) each chain advances by exactly that many
    original samples; ``K`` is then a cap and ``n_records`` the records made.
    ``step0`` is a scalar or one first step index per chain.
    ``follow = (actions, multiplicities)`` ([C, K] each) replays given
    records: ``action`` / ``M`` then hold the oracle's own decisions, ``cls``
    the RP_* class of each given record, and every other output is derived
    along the given trajectory (see ``replay``).
    """
    is_int, Qc = _as_q(Q)
    N = Qc.shape[0]
    C = num_chains
    cids = np.arange(C, dtype=np.uint32) if chain_ids is None else np.ascontiguousarray(chain_ids, dtype=np.uint32)
    betas = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, dtype=np.float64), (C,)))
    if x0 is None:
        if init == "zero":
            x0 = np.zeros((C, N), dtype=np.uint8)
        elif init == "random":
            x0 = np.stack([random_state(seed, int(c), N) for c in cids])
        else:
            raise ValueError(init)
    x0 = np.ascontiguousarray(np.broadcast_to(np.asarray(x0, dtype=np.uint8), (C, N)))
    r = RunResult()
    if log:
        r.action = np.zeros((C, K), dtype=np.int32)
        r.M = np.zeros((C, K), dtype=np.int64)
        r.E = np.zeros((C, K), dtype=np.int64 if is_int else np.float64)
        r.p = np.zeros((C, K))
        r.q = np.zeros((C, K))
        r.tmargin = np.zeros((C, K))
        r.w = np.zeros((C, K))
    r.x = np.zeros((C, N), dtype=np.uint8)
    r.h = np.zeros((C, N), dtype=np.int64 if is_int else np.float64)
    r.E_final = np.zeros(C, dtype=np.int64 if is_int else np.float64)
    Ef_dummy = np.zeros(C)
    r.L = np.zeros(C, dtype=np.int64)
    r.sub = np.zeros(C, dtype=np.int64)
    r.flips = np.zeros(C, dtype=np.int64)
    r.stays = np.zeros(C, dtype=np.int64)
    r.saturated = np.zeros(C, dtype=np.int64)
    if hist:
        if N > 24:
            raise ValueError("histograms need N <= 24")
        r.hist_w = np.zeros(1 << N, dtype=np.uint64)
        r.hist_v = np.zeros(1 << N, dtype=np.uint64)
        r.hist_rb = np.zeros(1 << N, dtype=np.float64)
    a = _RunArgs()
    a.N, a.is_int, a.layout = N, is_int, layout
    a.Qi = Qc.ctypes.data if is_int else None
    a.Qf = None if is_int else Qc.ctypes.data
    a.mode, a.n, a.L0, a.seed = mode, (N if mode == MODE_RF else n), L0, seed
    step0s = None
    if np.ndim(step0) > 0:
        step0s = np.ascontiguousarray(step0, dtype=np.int64)
        step0 = 0
    a.num_chains, a.chain_ids, a.betas, a.x0, a.K, a.step0 = C, cids.ctypes.data, betas.ctypes.data, x0.ctypes.data, K, int(step0)
    a.log_action = _ptr(r.action)
    a.log_M = _ptr(r.M)
    a.log_Ei = _ptr(r.E) if (log and is_int) else None
    a.log_Ef = _ptr(r.E) if (log and not is_int) else None
    a.log_p, a.log_q, a.log_tmargin = _ptr(r.p), _ptr(r.q), _ptr(r.tmargin)
    a.x_final = _ptr(r.x)
    a.hi_final = _ptr(r.h) if is_int else None
    a.hf_final = None if is_int else _ptr(r.h)
    a.Ei_final = _ptr(r.E_final) if is_int else None
    a.Ef_final = _ptr(Ef_dummy) if is_int else _ptr(r.E_final)
    a.L_final, a.sub_final = _ptr(r.L), _ptr(r.sub)
    a.hist_w, a.hist_v, a.hist_from = _ptr(r.hist_w), _ptr(r.hist_v), hist_from
    a.n_flips, a.n_stays, a.n_saturated = _ptr(r.flips), _ptr(r.stays), _ptr(r.saturated)
    a.temperature = temperature
    r.x_best = np.zeros((C, N), dtype=np.uint8)
    r.E_best = np.zeros(C, dtype=np.int64 if is_int else np.float64)
    Eb_dummy = np.zeros(C, dtype=np.float64 if is_int else np.int64)
    a.x_best = _ptr(r.x_best)
    a.Ei_best = _ptr(r.E_best) if is_int else _ptr(Eb_dummy)
    a.Ef_best = _ptr(Eb_dummy) if is_int else _ptr(r.E_best)
    a.orig_time = orig_time
    r.n_records = np.zeros(C, dtype=np.int64)
    a.n_records = _ptr(r.n_records)
    a.step0s = _ptr(step0s)
    a.log_w, a.hist_rb = _ptr(r.w), _ptr(r.hist_rb)
    if follow is not None:
        fa = np.ascontiguousarray(follow[0], dtype=np.int32)
        fm = np.ascontiguousarray(follow[1], dtype=np.int64)
        if fa.shape != (C, K) or fm.shape != (C, K):
            raise ValueError(f"follow arrays must be [{C}, {K}]")
        r.cls = np.zeros((C, K), dtype=np.int32)
        a.rp_action, a.rp_M, a.rp_class, a.rp_tol = fa.ctypes.data, fm.ctypes.data, r.cls.ctypes.data, follow_tol
    rc = (lib_handle or lib()).orc_run(ctypes.byref(a))
    if rc != 0:
        raise ValueError(f"oracle run rejected its arguments (code {rc})")
    return r


def replay(Q: np.ndarray, beta, mode: int, actions: np.ndarray, multiplicities: np.ndarray, *, tol: float,
           **kw) -> RunResult:
    """Replay mode: follow another implementation's records.

    For each given record (action, M) of each chain the oracle derives, from
    its own state and its own Philox draws, dE, the weights, p, q and its own
    decision, classifies the given record against that decision (``cls``,
    RP_*) and continues from the given decision, so that every later record
    is derived along the given trajectory and nothing stops at a difference.
    A differing decision counts as a decision-boundary case only where the
    oracle's quotient q (against the budget L or an integer) or U2*S (against
    a running-sum end of the given choice) lies within the band that a
    relative difference ``tol`` in p can move it across; anything else is
    RP_MISMATCH.  ``E`` and ``p`` are the oracle's values along the
    trajectory, ``x``/``h``/``E_final`` its final state.  Other keywords as
    in ``run``."""
    actions = np.asarray(actions)
    K = actions.shape[1]
    return run(Q, beta, mode, K, follow=(actions, multiplicities), follow_tol=tol, **kw)


class _ContArgs(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("mu0", ctypes.c_double), ("sigma", ctypes.c_double), ("pairs", ctypes.c_int32),
        ("L0", ctypes.c_int64), ("seed", ctypes.c_uint64), ("num_chains", ctypes.c_int32),
        ("chain_ids", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("K", ctypes.c_int64),
        ("log_action", ctypes.c_void_p), ("log_M", ctypes.c_void_p), ("log_lp", ctypes.c_void_p),
        ("log_p", ctypes.c_void_p), ("log_q", ctypes.c_void_p), ("log_tmargin", ctypes.c_void_p),
        ("log_w", ctypes.c_void_p), ("log_x", ctypes.c_void_p),
        ("x_final", ctypes.c_void_p), ("L_final", ctypes.c_void_p), ("set_final", ctypes.c_void_p),
        ("n_flips", ctypes.c_void_p), ("n_stays", ctypes.c_void_p), ("sums", ctypes.c_void_p),
        ("rp_action", ctypes.c_void_p), ("rp_M", ctypes.c_void_p), ("rp_class", ctypes.c_void_p),
        ("rp_tol", ctypes.c_double),
    ]


@dataclass
class ContResult:
    action: Optional[np.ndarray] = None   # [C, K] neighbour index or STAY
    M: Optional[np.ndarray] = None
    E: Optional[np.ndarray] = None        # log pi of the record's state (named E for the shared comparisons)
    p: Optional[np.ndarray] = None
    q: Optional[np.ndarray] = None
    tmargin: Optional[np.ndarray] = None
    w: Optional[np.ndarray] = None
    xs: Optional[np.ndarray] = None       # [C, K, dim] record states (log_states=True)
    x: Optional[np.ndarray] = None        # [C, dim] final states
    L: Optional[np.ndarray] = None
    set: Optional[np.ndarray] = None
    flips: Optional[np.ndarray] = None
    stays: Optional[np.ndarray] = None
    sums: Optional[np.ndarray] = None     # [C, 2, 4 dim + 1]
    cls: Optional[np.ndarray] = None      # replay: RP_* class of each followed record


def cont_run(x0: np.ndarray, K: int, *, mu0: float = 9.0, sigma: float = 0.1, pairs: int = 25, L0: int = 1000,
             seed: int = 0, chain_ids=None, log: bool = True, log_states: bool = False,
             lib_handle: Optional[ctypes.CDLL] = None, follow=None, follow_tol: float = 0.0) -> ContResult:
    """Continuous Unbiased PNS (Alg 7) on the donut target from states x0
    [C, dim] for K records per chain (see orc_cont_run).  ``follow`` and
    ``follow_tol`` replay given records as in ``run`` / ``replay``."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    C, d = x0.shape
    cids = np.arange(C, dtype=np.uint32) if chain_ids is None else np.ascontiguousarray(chain_ids, dtype=np.uint32)
    r = ContResult()
    if log:
        r.action = np.zeros((C, K), np.int32)
        r.M = np.zeros((C, K), np.int64)
        r.E = np.zeros((C, K))
        r.p = np.zeros((C, K))
        r.q = np.zeros((C, K))
        r.tmargin = np.zeros((C, K))
        r.w = np.zeros((C, K))
    if log_states:
        r.xs = np.zeros((C, K, d))
    r.x = np.zeros((C, d))
    r.L = np.zeros(C, np.int64)
    r.set = np.zeros(C, np.int64)
    r.flips = np.zeros(C, np.int64)
    r.stays = np.zeros(C, np.int64)
    r.sums = np.zeros((C, 2, 4 * d + 1))
    a = _ContArgs()
    a.dim, a.mu0, a.sigma, a.pairs, a.L0, a.seed = d, mu0, sigma, pairs, L0, seed
    a.num_chains, a.chain_ids, a.x0, a.K = C, cids.ctypes.data, x0.ctypes.data, K
    a.log_action, a.log_M, a.log_lp, a.log_p = _ptr(r.action), _ptr(r.M), _ptr(r.E), _ptr(r.p)
    a.log_q, a.log_tmargin, a.log_w, a.log_x = _ptr(r.q), _ptr(r.tmargin), _ptr(r.w), _ptr(r.xs)
    a.x_final, a.L_final, a.set_final = _ptr(r.x), _ptr(r.L), _ptr(r.set)
    a.n_flips, a.n_stays, a.sums = _ptr(r.flips), _ptr(r.stays), _ptr(r.sums)
    if follow is not None:
        fa = np.ascontiguousarray(follow[0], dtype=np.int32)
        fm = np.ascontiguousarray(follow[1], dtype=np.int64)
        if fa.shape != (C, K) or fm.shape != (C, K):
            raise ValueError(f"follow arrays must be [{C}, {K}]")
        r.cls = np.zeros((C, K), dtype=np.int32)
        a.rp_action, a.rp_M, a.rp_class, a.rp_tol = fa.ctypes.data, fm.ctypes.data, r.cls.ctypes.data, follow_tol
    rc = (lib_handle or lib()).orc_cont_run(ctypes.byref(a))
    if rc != 0:
        raise ValueError(f"oracle continuous run rejected its arguments (code {rc})")
    return r


def cont_offsets(seed: int, chain: int, set_index: int, pairs: int, dim: int) -> np.ndarray:
    """Offset vectors [pairs, dim] of partial neighbor set `set_index`."""
    out = np.zeros((pairs, dim))
    lib().orc_cont_offsets(seed, chain, set_index, pairs, dim, out.ctypes.data)
    return out


def expected_multiplicity(p: float, L: int = -1, lib_handle: Optional[ctypes.CDLL] = None) -> float:
    """E[min(1 + G, L)] for G geometric (failures) with success probability
    p, the mean multiplicity of a record (Thm 3 (2)); L < 0: no budget."""
    return float((lib_handle or lib()).orc_expected_multiplicity(float(p), int(L)))


def pt_round(energies: np.ndarray, betas: np.ndarray, ladder: np.ndarray, T: int, seed: int, round_: int,
             lib_handle: Optional[ctypes.CDLL] = None):
    """One parallel-tempering swap round (see orc_pt_round); ``betas`` and
    ``ladder`` (int32 [groups * T]) are updated in place.  Returns the
    accepted flags [groups * T]."""
    E = np.ascontiguousarray(energies)
    is_int = np.issubdtype(E.dtype, np.integer)
    Ei = E.astype(np.int64) if is_int else None
    Ef = None if is_int else E.astype(np.float64)
    assert betas.dtype == np.float64 and betas.flags["C_CONTIGUOUS"]
    assert ladder.dtype == np.int32 and ladder.flags["C_CONTIGUOUS"]
    groups = len(betas) // T
    acc = np.zeros(groups * T, dtype=np.int32)
    L = lib_handle or lib()
    if lib_handle is not None:
        _declare(L)
    rc = L.orc_pt_round(groups, T, int(is_int), _ptr(Ei), _ptr(Ef), betas.ctypes.data, ladder.ctypes.data,
                        seed, round_, acc.ctypes.data)
    if rc != 0:
        raise ValueError("bad pt_round arguments")
    return acc
