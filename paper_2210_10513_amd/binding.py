"""Thin ctypes binding of libpns.so (declarations in include/pns.h).

Functions keep the C names (``pns_create``, ``pns_run``, ``pns_read`` ...) and
only marshal arguments: numpy arrays and torch tensors (host or device) are
passed as raw pointers, every step of the sampler runs in the library's HIP
kernels.  There is no fallback: if the library is missing or fails to load,
importing this module raises.

``Sampler`` (one problem) and ``BatchSampler`` (several problems of uneven N
in one context) are small convenience wrappers that own a context and return
numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libpns.so")

PNS_OK, PNS_EINVAL, PNS_ENOMEM, PNS_EDEVICE, PNS_EUNSUPPORTED = 0, 1, 2, 3, 4
PNS_MODE_RF, PNS_MODE_BASIC, PNS_MODE_UNBIASED_SYS, PNS_MODE_UNBIASED_RAND = 0, 1, 2, 3
PNS_I16, PNS_I32, PNS_F32 = 0, 1, 2
PNS_SYMMETRIC, PNS_UPPER = 0, 1
PNS_INIT_ZERO, PNS_INIT_RANDOM, PNS_INIT_GIVEN = 0, 1, 2
PNS_LAUNCH_PLAIN, PNS_LAUNCH_PERSISTENT, PNS_LAUNCH_GRAPH = 0, 1, 2
PNS_STAY = -1

MODES = {"rf": PNS_MODE_RF, "basic": PNS_MODE_BASIC, "unbiased_sys": PNS_MODE_UNBIASED_SYS,
         "unbiased_rand": PNS_MODE_UNBIASED_RAND}
LAUNCHES = {"plain": PNS_LAUNCH_PLAIN, "persistent": PNS_LAUNCH_PERSISTENT, "graph": PNS_LAUNCH_GRAPH}
INITS = {"zero": PNS_INIT_ZERO, "random": PNS_INIT_RANDOM, "given": PNS_INIT_GIVEN}
LAYOUTS = {"symmetric": PNS_SYMMETRIC, "upper": PNS_UPPER}

EXPORTS = ["pns_opts_default", "pns_create", "pns_run", "pns_read", "pns_read_current", "pns_field_type",
           "pns_read_log", "pns_read_hist", "pns_hist_clear", "pns_read_snapshots", "pns_stats", "pns_sync",
           "pns_destroy", "pns_tile", "pns_last_error", "pns_version", "pns_create_batch", "pns_autotune",
           "pns_chain_offsets", "pns_num_problems", "pns_problem_info_get", "pns_moments", "pns_snapshot_moments",
           "pns_log_partition", "pns_set_q", "pns_snapshots_clear", "pns_optimize", "pns_read_best",
           "pns_adopt_best", "pns_run_original", "pns_pt_swap", "pns_read_betas", "pns_read_ladder",
           "pns_moments_f64", "pns_read_rb_weights", "pns_snapshot_moments_rb", "pns_cont_opts_default",
           "pns_cont_create", "pns_cont_run", "pns_cont_read", "pns_cont_read_log", "pns_cont_read_sums",
           "pns_cont_clear_sums", "pns_cont_stats", "pns_cont_sync", "pns_cont_destroy", "pns_save", "pns_load", "pns_profile",
           "pns_profile_read", "pns_class_of_chain", "pns_moments_noalloc", "pns_refresh", "pns_logz_grad"]


class pns_class_profile(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32), ("groups", ctypes.c_int32), ("flavour", ctypes.c_int32),
        ("chains", ctypes.c_int32), ("N_min", ctypes.c_int32), ("N_max", ctypes.c_int32),
        ("launches", ctypes.c_int64), ("kernel_ms", ctypes.c_double), ("flips", ctypes.c_int64),
        ("records", ctypes.c_int64), ("row_bytes", ctypes.c_double),
    ]


class pns_opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32), ("num_chains", ctypes.c_int32),
        ("betas", ctypes.c_void_p), ("L0", ctypes.c_int64), ("seed", ctypes.c_uint64),
        ("chain_id_base", ctypes.c_uint32), ("init", ctypes.c_int32), ("x0", ctypes.c_void_p),
        ("launch", ctypes.c_int32), ("chunk", ctypes.c_int32), ("block", ctypes.c_int32),
        ("groups", ctypes.c_int32), ("stream", ctypes.c_void_p), ("log_capacity", ctypes.c_int64),
        ("hist", ctypes.c_int32), ("snapshot_every", ctypes.c_int32), ("snapshot_capacity", ctypes.c_int32),
        ("autotune", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7),
    ]


class pns_cont_opts(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("pairs", ctypes.c_int32), ("mu0", ctypes.c_double), ("sigma", ctypes.c_double),
        ("L0", ctypes.c_int64), ("seed", ctypes.c_uint64), ("num_chains", ctypes.c_int32),
        ("chain_id_base", ctypes.c_uint32), ("x0", ctypes.c_void_p), ("log_capacity", ctypes.c_int64),
        ("stream", ctypes.c_void_p), ("reserved", ctypes.c_int32 * 8),
    ]


class pns_problem(ctypes.Structure):
    _fields_ = [("Q", ctypes.c_void_p), ("N", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("subset_size", ctypes.c_int32), ("num_chains", ctypes.c_int32), ("L0", ctypes.c_int64),
                ("betas", ctypes.c_void_p), ("beta", ctypes.c_double)]


class pns_problem_info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("subset_size", ctypes.c_int32), ("block", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("chain_begin", ctypes.c_int32), ("num_chains", ctypes.c_int32),
                ("flavour", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class pns_tune(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("groups", ctypes.c_int32), ("subset_size", ctypes.c_int32),
                ("trials", ctypes.c_int32), ("records_per_s", ctypes.c_double), ("flips_per_s", ctypes.c_double)]


class pns_chain_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("flips", ctypes.c_int64), ("stays", ctypes.c_int64),
                ("saturated", ctypes.c_int64), ("sum_M", ctypes.c_double), ("anomalies", ctypes.c_int64)]


class PNSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pns error {code}: {msg}")
        self.code = code


def _load() -> ctypes.CDLL:
    # PyTorch-ROCm ships its own HIP runtime under the same soname; loading it
    # first makes libpns.so bind to that one runtime, so torch's streams and
    # device pointers are the library's too (a second runtime in the process
    # would leave torch without a device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_10513_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.pns_opts_default.argtypes = [ctypes.POINTER(pns_opts)]
    L.pns_opts_default.restype = None
    L.pns_create.argtypes = [ctypes.POINTER(vp), vp, i32, dbl, i32, i32, ctypes.POINTER(pns_opts)]
    L.pns_run.argtypes = [vp, i64]
    L.pns_read.argtypes = [vp, vp, vp, vp]
    L.pns_read_current.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pns_field_type.argtypes = [vp]
    L.pns_read_log.argtypes = [vp, vp, vp, vp, vp]
    L.pns_read_hist.argtypes = [vp, vp, vp]
    L.pns_hist_clear.argtypes = [vp]
    L.pns_read_snapshots.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i32)]
    L.pns_stats.argtypes = [vp, ctypes.POINTER(pns_chain_stats)]
    L.pns_sync.argtypes = [vp]
    L.pns_destroy.argtypes = [vp]
    L.pns_tile.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.pns_last_error.argtypes = []
    L.pns_last_error.restype = ctypes.c_char_p
    L.pns_version.argtypes = []
    L.pns_version.restype = ctypes.c_char_p
    L.pns_create_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(pns_problem), i32, ctypes.POINTER(pns_opts)]
    L.pns_autotune.argtypes = [vp, i32, dbl, i32, i32, ctypes.POINTER(pns_opts), i32, ctypes.POINTER(pns_tune)]
    L.pns_chain_offsets.argtypes = [vp, vp]
    L.pns_num_problems.argtypes = [vp]
    L.pns_problem_info_get.argtypes = [vp, i32, ctypes.POINTER(pns_problem_info)]
    L.pns_moments.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp]
    L.pns_snapshot_moments.argtypes = [vp, i32, vp, vp]
    L.pns_log_partition.argtypes = [vp, i32, i32, i32, dbl, vp, vp]
    L.pns_set_q.argtypes = [vp, i32, vp]
    L.pns_snapshots_clear.argtypes = [vp]
    L.pns_optimize.argtypes = [vp, i64, dbl]
    L.pns_read_best.argtypes = [vp, vp, vp]
    L.pns_adopt_best.argtypes = [vp]
    L.pns_run_original.argtypes = [vp, i64]
    L.pns_pt_swap.argtypes = [vp, i32, i64, vp]
    L.pns_read_betas.argtypes = [vp, vp]
    L.pns_read_ladder.argtypes = [vp, vp]
    L.pns_moments_noalloc.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp]
    L.pns_refresh.argtypes = [vp]
    L.pns_profile.argtypes = [vp, i32]
    L.pns_profile_read.argtypes = [vp, ctypes.POINTER(pns_class_profile), i32, ctypes.POINTER(i32)]
    L.pns_class_of_chain.argtypes = [vp, vp]
    L.pns_save.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
    L.pns_load.argtypes = [vp, vp, i64]
    L.pns_moments_f64.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp]
    L.pns_read_rb_weights.argtypes = [vp, vp, vp, vp]
    L.pns_snapshot_moments_rb.argtypes = [vp, i32, vp, vp]
    L.pns_logz_grad.argtypes = [vp, i32, dbl, i32, vp, vp]
    L.pns_cont_opts_default.argtypes = [ctypes.POINTER(pns_cont_opts)]
    L.pns_cont_opts_default.restype = None
    L.pns_cont_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(pns_cont_opts)]
    L.pns_cont_run.argtypes = [vp, i64]
    L.pns_cont_read.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pns_cont_read_log.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pns_cont_read_sums.argtypes = [vp, vp]
    L.pns_cont_clear_sums.argtypes = [vp]
    L.pns_cont_stats.argtypes = [vp, vp, vp]
    L.pns_cont_sync.argtypes = [vp]
    L.pns_cont_destroy.argtypes = [vp]
    for name in ("pns_create", "pns_run", "pns_read", "pns_read_current", "pns_field_type", "pns_read_log",
                 "pns_read_hist", "pns_hist_clear", "pns_read_snapshots", "pns_stats", "pns_sync", "pns_destroy",
                 "pns_tile", "pns_create_batch", "pns_autotune", "pns_chain_offsets", "pns_num_problems",
                 "pns_problem_info_get", "pns_moments", "pns_snapshot_moments", "pns_log_partition", "pns_set_q",
                 "pns_snapshots_clear", "pns_optimize", "pns_read_best", "pns_adopt_best", "pns_run_original",
                 "pns_pt_swap", "pns_read_betas", "pns_read_ladder", "pns_moments_f64", "pns_read_rb_weights",
                 "pns_snapshot_moments_rb", "pns_cont_create", "pns_cont_run", "pns_cont_read", "pns_cont_read_log",
                 "pns_cont_read_sums", "pns_cont_clear_sums", "pns_cont_stats", "pns_cont_sync", "pns_cont_destroy",
                 "pns_save", "pns_load", "pns_profile", "pns_profile_read", "pns_class_of_chain",
                 "pns_moments_noalloc", "pns_refresh"):
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(rc: int) -> None:
    if rc != PNS_OK:
        raise PNSError(rc, lib.pns_last_error().decode())


def _addr(a) -> Optional[int]:
    """Raw pointer of a numpy array or torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays passed to the library must be C-contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensors passed to the library must be contiguous")
        return a.data_ptr()
    raise TypeError(f"cannot pass {type(a)} to the library")


# ---- C-named wrappers (argument marshalling only) ----

def pns_opts_default() -> pns_opts:
    o = pns_opts()
    lib.pns_opts_default(ctypes.byref(o))
    return o


def pns_create(Q, N: int, beta: float, subset_size: int, mode: int, opts: Optional[pns_opts] = None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(lib.pns_create(ctypes.byref(ctx), _addr(Q), N, beta, subset_size, mode,
                          ctypes.byref(opts) if opts is not None else None))
    return ctx


def pns_run(ctx, steps: int) -> None:
    _check(lib.pns_run(ctx, steps))


def pns_read(ctx, states=None, multiplicities=None, energies=None) -> None:
    _check(lib.pns_read(ctx, _addr(states), _addr(multiplicities), _addr(energies)))


def pns_read_current(ctx, states=None, energies=None, fields=None, L=None, set_index=None, step=None) -> None:
    _check(lib.pns_read_current(ctx, _addr(states), _addr(energies), _addr(fields), _addr(L), _addr(set_index),
                                _addr(step)))


def pns_field_type(ctx) -> int:
    return int(lib.pns_field_type(ctx))


def pns_read_log(ctx, actions=None, multiplicities=None, energies=None, p=None) -> None:
    _check(lib.pns_read_log(ctx, _addr(actions), _addr(multiplicities), _addr(energies), _addr(p)))


def pns_read_hist(ctx, hist_weighted=None, hist_visits=None) -> None:
    _check(lib.pns_read_hist(ctx, _addr(hist_weighted), _addr(hist_visits)))


def pns_hist_clear(ctx) -> None:
    _check(lib.pns_hist_clear(ctx))


def pns_read_snapshots(ctx, states=None, multiplicities=None, energies=None) -> int:
    cnt = ctypes.c_int32()
    _check(lib.pns_read_snapshots(ctx, _addr(states), _addr(multiplicities), _addr(energies), ctypes.byref(cnt)))
    return cnt.value


def pns_stats(ctx, num_chains: int):
    arr = (pns_chain_stats * num_chains)()
    _check(lib.pns_stats(ctx, arr))
    return arr


def pns_sync(ctx) -> None:
    _check(lib.pns_sync(ctx))


def pns_destroy(ctx) -> None:
    _check(lib.pns_destroy(ctx))


def pns_tile(ctx):
    b, g = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.pns_tile(ctx, ctypes.byref(b), ctypes.byref(g)))
    return b.value, g.value


def pns_create_batch(problems, mode: int, opts: Optional[pns_opts] = None) -> ctypes.c_void_p:
    """``problems`` is a sequence of ``pns_problem`` (kept alive by the caller)."""
    arr = (pns_problem * len(problems))(*problems)
    ctx = ctypes.c_void_p()
    _check(lib.pns_create_batch(ctypes.byref(ctx), len(problems), arr, mode,
                                ctypes.byref(opts) if opts is not None else None))
    return ctx


def pns_autotune(Q, N: int, beta: float, subset_size: int, mode: int, opts: Optional[pns_opts] = None,
                 trial_steps: int = 64) -> pns_tune:
    out = pns_tune()
    _check(lib.pns_autotune(_addr(Q), N, beta, subset_size, mode, ctypes.byref(opts) if opts is not None else None,
                            trial_steps, ctypes.byref(out)))
    return out


def pns_chain_offsets(ctx, num_chains: int) -> np.ndarray:
    off = np.zeros(num_chains + 1, np.int64)
    _check(lib.pns_chain_offsets(ctx, off.ctypes.data))
    return off


def pns_num_problems(ctx) -> int:
    return int(lib.pns_num_problems(ctx))


def pns_problem_info_get(ctx, p: int) -> pns_problem_info:
    info = pns_problem_info()
    _check(lib.pns_problem_info_get(ctx, p, ctypes.byref(info)))
    return info


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    return stream if isinstance(stream, int) else stream.cuda_stream


def pns_moments(X, m, G, *, N: Optional[int] = None, ldx: Optional[int] = None, stream=None, sum_m=None):
    """G[:] = X^T diag(m) X.  X [K, ldx] uint8, m [K] int64, G [N, N]
    float64 (numpy arrays or torch tensors, host or device).  Returns sum(m)
    as a float, or writes it into ``sum_m`` (a one-element float64 array or
    tensor, host or device) and returns None."""
    K = int(X.shape[0])
    ld = int(X.shape[1]) if ldx is None else ldx
    n = int(G.shape[0]) if N is None else N
    if sum_m is not None:
        _check(lib.pns_moments(_addr(X), ld, _addr(m), K, n, _addr(G), _addr(sum_m), _stream_handle(stream)))
        return None
    sm = np.zeros(1, np.float64)
    _check(lib.pns_moments(_addr(X), ld, _addr(m), K, n, _addr(G), sm.ctypes.data, _stream_handle(stream)))
    return float(sm[0])


def pns_moments_f64(X, w, G, *, N: Optional[int] = None, ldx: Optional[int] = None, stream=None, sum_w=None):
    """G[:] = X^T diag(w) X with w [K] float64; otherwise like pns_moments."""
    K = int(X.shape[0])
    ld = int(X.shape[1]) if ldx is None else ldx
    n = int(G.shape[0]) if N is None else N
    if sum_w is not None:
        _check(lib.pns_moments_f64(_addr(X), ld, _addr(w), K, n, _addr(G), _addr(sum_w), _stream_handle(stream)))
        return None
    sm = np.zeros(1, np.float64)
    _check(lib.pns_moments_f64(_addr(X), ld, _addr(w), K, n, _addr(G), sm.ctypes.data, _stream_handle(stream)))
    return float(sm[0])


def pns_snapshot_moments(ctx, problem: int, G, sum_m=None, *, rb: bool = False):
    """Moments of the snapshots of one problem; like pns_moments.  With
    ``rb`` the weights are the expected multiplicities (pns_read_rb_weights)."""
    fn = lib.pns_snapshot_moments_rb if rb else lib.pns_snapshot_moments
    if sum_m is not None:
        _check(fn(ctx, problem, _addr(G), _addr(sum_m)))
        return None
    sm = np.zeros(1, np.float64)
    _check(fn(ctx, problem, _addr(G), sm.ctypes.data))
    return float(sm[0])


def pns_logz_grad(ctx, problem: int, beta: float, grad, sum_w, *, rb: bool = False) -> None:
    """-beta * G / sum_w of one problem's snapshots into device buffers
    (grad [N][N] FP64, sum_w [1] FP64), queued on the context's stream."""
    _check(lib.pns_logz_grad(ctx, problem, beta, 1 if rb else 0, _addr(grad), _addr(sum_w)))


def pns_read_rb_weights(ctx, log_w=None, snap_w=None, hist_rb=None) -> None:
    _check(lib.pns_read_rb_weights(ctx, _addr(log_w), _addr(snap_w), _addr(hist_rb)))


def pns_log_partition(Q, beta: float, *, layout: int = PNS_SYMMETRIC, stream=None) -> float:
    """log sum_x exp(-beta x^T Q x) by enumeration on the device (N <= 32)."""
    if hasattr(Q, "data_ptr"):
        import torch
        dt = {torch.int16: PNS_I16, torch.int32: PNS_I32, torch.float32: PNS_F32}[Q.dtype]
        Qk = Q.contiguous()
    else:
        Qk = np.ascontiguousarray(Q)
        dt = _DTYPES[Qk.dtype]
    out = np.zeros(1, np.float64)
    _check(lib.pns_log_partition(_addr(Qk), int(Qk.shape[0]), dt, layout, float(beta), out.ctypes.data,
                                 _stream_handle(stream)))
    return float(out[0])


def pns_set_q(ctx, problem: int, Q) -> None:
    _check(lib.pns_set_q(ctx, problem, _addr(Q)))


def pns_snapshots_clear(ctx) -> None:
    _check(lib.pns_snapshots_clear(ctx))


def pns_optimize(ctx, steps: int, temperature: float = 1.0) -> None:
    _check(lib.pns_optimize(ctx, steps, float(temperature)))


def pns_read_best(ctx, states=None, energies=None) -> None:
    _check(lib.pns_read_best(ctx, _addr(states), _addr(energies)))


def pns_adopt_best(ctx) -> None:
    _check(lib.pns_adopt_best(ctx))


def pns_run_original(ctx, original_steps: int) -> None:
    _check(lib.pns_run_original(ctx, original_steps))


def pns_pt_swap(ctx, temps: int, round_: int, accepted=None) -> None:
    _check(lib.pns_pt_swap(ctx, temps, round_, _addr(accepted)))


def pns_read_betas(ctx, betas) -> None:
    _check(lib.pns_read_betas(ctx, _addr(betas)))


def pns_read_ladder(ctx, ladder) -> None:
    _check(lib.pns_read_ladder(ctx, _addr(ladder)))


def pns_moments_noalloc(X, m, G, sum_m=None, *, N: Optional[int] = None, ldx: Optional[int] = None,
                        stream=None) -> None:
    """G = X^T diag(m) X into device tensors without any allocation (the
    library's static per-GPU workspace); X [K][ldx] uint8, m [K] int64,
    G [N][N] float64 and sum_m [1] float64 (or None) must be device tensors."""
    K = int(X.shape[0])
    ld = int(X.shape[1]) if ldx is None else ldx
    n = int(G.shape[0]) if N is None else N
    _check(lib.pns_moments_noalloc(_addr(X), ld, _addr(m), K, n, _addr(G), _addr(sum_m), _stream_handle(stream)))


def pns_refresh(ctx) -> None:
    _check(lib.pns_refresh(ctx))


def pns_profile(ctx, enable: bool = True) -> None:
    _check(lib.pns_profile(ctx, 1 if enable else 0))


def pns_profile_read(ctx):
    """Per launch class: tile, flavour, chains, N range, launches, summed
    kernel time (HIP events on the class's stream), flips, records and
    algorithmic row bytes since pns_profile."""
    n = ctypes.c_int32(0)
    _check(lib.pns_profile_read(ctx, None, 0, ctypes.byref(n)))
    arr = (pns_class_profile * max(1, n.value))()
    _check(lib.pns_profile_read(ctx, arr, n.value, ctypes.byref(n)))
    return [{f: getattr(arr[i], f) for f, _ in pns_class_profile._fields_} for i in range(n.value)]


def pns_class_of_chain(ctx, num_chains: int) -> np.ndarray:
    out = np.zeros(num_chains, np.int32)
    _check(lib.pns_class_of_chain(ctx, out.ctypes.data))
    return out


def pns_save(ctx, buf=None) -> int:
    """Checkpoint size in bytes (buf None), or write the checkpoint into buf
    (a host or device buffer of at least that size) and return its size."""
    size = ctypes.c_int64(0)
    cap = 0 if buf is None else (buf.nbytes if hasattr(buf, "nbytes") else buf.numel() * buf.element_size())
    _check(lib.pns_save(ctx, _addr(buf), cap, ctypes.byref(size)))
    return size.value


def pns_load(ctx, buf, size: int) -> None:
    _check(lib.pns_load(ctx, _addr(buf), size))


def pns_last_error() -> str:
    return lib.pns_last_error().decode()


def pns_version() -> str:
    return lib.pns_version().decode()


# ---- convenience wrapper ----

_DTYPES = {np.dtype(np.int16): PNS_I16, np.dtype(np.int32): PNS_I32, np.dtype(np.float32): PNS_F32}
_FIELD_DTYPES = {0: np.int32, 1: np.int64, 2: np.float64}


class Sampler:
    """One sampler context.  ``Q`` is a numpy array or torch tensor of int16,
    int32 or float32 (host or device); results come back as numpy arrays."""

    def __init__(self, Q, beta=1.0, subset_size: int = 0, mode="rf", *, num_chains: int = 1, L0: int = 100,
                 seed: int = 0, init="zero", x0=None, layout="symmetric", launch="persistent", chunk: int = 0,
                 block: int = 0, groups: int = 0, stream=None, log_capacity: int = 0, hist: bool = False,
                 snapshot_every: int = 0, snapshot_capacity: int = 0, chain_id_base: int = 0,
                 autotune: bool = False):
        if hasattr(Q, "data_ptr"):
            import torch
            dt = {torch.int16: PNS_I16, torch.int32: PNS_I32, torch.float32: PNS_F32}[Q.dtype]
            self.N = int(Q.shape[0])
            self._Q = Q.contiguous()
        else:
            Qa = np.ascontiguousarray(Q)
            if Qa.dtype not in _DTYPES:
                raise TypeError("Q must be int16, int32 or float32")
            dt = _DTYPES[Qa.dtype]
            self.N = int(Qa.shape[0])
            self._Q = Qa
        self.num_chains = num_chains
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        o = pns_opts_default()
        o.dtype = dt
        o.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
        o.num_chains = num_chains
        betas = np.broadcast_to(np.asarray(beta, dtype=np.float64), (num_chains,)).copy()
        self._betas = betas
        o.betas = betas.ctypes.data
        o.L0 = L0
        o.seed = seed
        o.chain_id_base = chain_id_base
        o.init = INITS[init] if isinstance(init, str) else int(init)
        if x0 is not None:
            o.init = PNS_INIT_GIVEN
            self._x0 = np.ascontiguousarray(np.broadcast_to(np.asarray(x0, dtype=np.uint8), (num_chains, self.N)))
            o.x0 = self._x0.ctypes.data
        o.launch = LAUNCHES[launch] if isinstance(launch, str) else int(launch)
        o.chunk = chunk
        o.block = block
        o.groups = groups
        if stream is not None:
            o.stream = stream if isinstance(stream, int) else stream.cuda_stream
        o.log_capacity = log_capacity
        o.hist = 1 if hist else 0
        o.snapshot_every = snapshot_every
        o.snapshot_capacity = snapshot_capacity
        o.autotune = 1 if autotune else 0
        self.log_capacity = log_capacity
        self.snapshot_capacity = snapshot_capacity
        self.snapshot_every = snapshot_every
        self.hist = bool(hist)
        self.ctx = pns_create(self._Q, self.N, float(betas[0]), subset_size, self.mode, o)

    def run(self, steps: int) -> "Sampler":
        pns_run(self.ctx, steps)
        return self

    def sync(self) -> None:
        pns_sync(self.ctx)

    def read(self):
        C, N = self.num_chains, self.N
        s = np.zeros((C, N), np.uint8)
        m = np.zeros(C, np.int64)
        e = np.zeros(C, np.float64)
        pns_read(self.ctx, s, m, e)
        return s, m, e

    def read_current(self):
        C, N = self.num_chains, self.N
        s = np.zeros((C, N), np.uint8)
        e = np.zeros(C, np.float64)
        h = np.zeros((C, N), _FIELD_DTYPES[pns_field_type(self.ctx)])
        L = np.zeros(C, np.int64)
        sub = np.zeros(C, np.int64)
        k = np.zeros(C, np.int64)
        pns_read_current(self.ctx, s, e, h, L, sub, k)
        return {"x": s, "E": e, "h": h, "L": L, "sub": sub, "step": k}

    def read_log(self):
        C, K = self.num_chains, self.log_capacity
        a = np.zeros((C, K), np.int32)
        m = np.zeros((C, K), np.int64)
        e = np.zeros((C, K), np.float64)
        p = np.zeros((C, K), np.float64)
        pns_read_log(self.ctx, a, m, e, p)
        return {"action": a, "M": m, "E": e, "p": p}

    def read_hist(self):
        w = np.zeros(1 << self.N, np.uint64)
        v = np.zeros(1 << self.N, np.uint64)
        pns_read_hist(self.ctx, w, v)
        return w, v

    def hist_clear(self) -> None:
        pns_hist_clear(self.ctx)

    def read_snapshots(self):
        C, S, N = self.num_chains, self.snapshot_capacity, self.N
        x = np.zeros((C, S, N), np.uint8)
        m = np.zeros((C, S), np.int64)
        e = np.zeros((C, S), np.float64)
        cnt = pns_read_snapshots(self.ctx, x, m, e)
        return x, m, e, cnt

    def stats(self):
        arr = pns_stats(self.ctx, self.num_chains)
        return {k: np.array([getattr(s, k) for s in arr]) for k in ("steps", "flips", "stays", "saturated", "sum_M", "anomalies")}

    def set_q(self, Q) -> "Sampler":
        """New coefficient matrix (same N, dtype, layout); chains keep their
        states (warm start)."""
        if hasattr(Q, "data_ptr"):
            Qk = Q.contiguous()
        else:
            Qk = np.ascontiguousarray(Q)
        pns_set_q(self.ctx, 0, Qk)
        self._Q = Qk
        return self

    def optimize(self, steps: int, temperature: float = 1.0) -> "Sampler":
        """Optimization RF / PNS burn-in (Alg 9, 10) at temperature T."""
        pns_optimize(self.ctx, steps, temperature)
        return self

    def read_best(self):
        s = np.zeros((self.num_chains, self.N), np.uint8)
        e = np.zeros(self.num_chains, np.float64)
        pns_read_best(self.ctx, s, e)
        return s, e

    def adopt_best(self) -> "Sampler":
        pns_adopt_best(self.ctx)
        return self

    def run_original(self, original_steps: int) -> "Sampler":
        """Advance every chain by exactly this many original samples."""
        pns_run_original(self.ctx, original_steps)
        return self

    def pt_swap(self, temps: int, round_: int):
        """One tempering swap round; returns the accepted flags."""
        acc = np.zeros(self.num_chains, np.int32)
        pns_pt_swap(self.ctx, temps, round_, acc)
        return acc

    def betas(self):
        b = np.zeros(self.num_chains, np.float64)
        pns_read_betas(self.ctx, b)
        return b

    def ladder(self):
        l = np.zeros(self.num_chains, np.int32)
        pns_read_ladder(self.ctx, l)
        return l

    def refresh(self) -> "Sampler":
        """Recompute every chain's fields and energy from its state (pns_refresh)."""
        pns_refresh(self.ctx)
        return self

    def save(self) -> np.ndarray:
        """Checkpoint of every chain's state (pns_save) as a byte array."""
        buf = np.zeros(pns_save(self.ctx), np.uint8)
        pns_save(self.ctx, buf)
        return buf

    def load(self, buf) -> "Sampler":
        """Restore a checkpoint of an identically created sampler (pns_load)."""
        b = np.ascontiguousarray(buf, dtype=np.uint8)
        pns_load(self.ctx, b, b.nbytes)
        return self

    def snapshots_clear(self) -> "Sampler":
        pns_snapshots_clear(self.ctx)
        return self

    def snapshot_moments(self, G=None, *, rb: bool = False):
        """(G, sum_w): G = X^T diag(w) X over every stored snapshot, w the
        multiplicities M, or with ``rb`` their expected values given the
        records (Rao-Blackwell weights)."""
        if G is None:
            G = np.zeros((self.N, self.N), np.float64)
        sm = pns_snapshot_moments(self.ctx, 0, G, rb=rb)
        return G, sm

    def rb_weights(self):
        """Expected multiplicities of the records: {"log": [C, log_capacity]
        or None, "snap": [C, snapshot_capacity] or None, "hist": [2^N] or
        None}, whichever outputs the sampler keeps."""
        C = self.num_chains
        lw = np.zeros((C, self.log_capacity)) if self.log_capacity else None
        sw = np.zeros((C, self.snapshot_capacity)) if self.snapshot_every else None
        hw = np.zeros(1 << self.N) if self.hist else None
        pns_read_rb_weights(self.ctx, lw, sw, hw)
        return {"log": lw, "snap": sw, "hist": hw}

    def tile(self):
        return pns_tile(self.ctx)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            pns_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _as_q(Q):
    """(array kept alive, dtype code, N) of a numpy array or torch tensor."""
    if hasattr(Q, "data_ptr"):
        import torch
        dt = {torch.int16: PNS_I16, torch.int32: PNS_I32, torch.float32: PNS_F32}[Q.dtype]
        return Q.contiguous(), dt, int(Q.shape[0])
    Qa = np.ascontiguousarray(Q)
    if Qa.dtype not in _DTYPES:
        raise TypeError("Q must be int16, int32 or float32")
    return Qa, _DTYPES[Qa.dtype], int(Qa.shape[0])


class BatchSampler:
    """Several QUBO problems (possibly of different N) in one context.

    ``problems`` is a list of dicts with keys ``Q`` (required), ``beta``
    (scalar or one value per chain), ``num_chains``, ``subset_size`` (0: chosen
    by the autotuner in subset modes), ``L0`` (0: the context default) and
    ``layout``.  Per-chain results come back as lists with one entry per
    problem."""

    def __init__(self, problems, mode="rf", *, L0: int = 100, seed: int = 0, init="zero", x0=None,
                 launch="persistent", chunk: int = 0, stream=None, log_capacity: int = 0, snapshot_every: int = 0,
                 snapshot_capacity: int = 0, chain_id_base: int = 0, autotune: bool = False):
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        self._keep = []
        structs = []
        dtype = None
        for pr in problems:
            Qk, dt, N = _as_q(pr["Q"])
            if dtype is None:
                dtype = dt
            elif dt != dtype:
                raise TypeError("every problem of a batch must have the same Q dtype")
            c = int(pr.get("num_chains", 1))
            b = np.broadcast_to(np.asarray(pr.get("beta", 1.0), dtype=np.float64), (c,)).copy()
            self._keep += [Qk, b]
            lay = pr.get("layout", "symmetric")
            structs.append(pns_problem(Q=_addr(Qk), N=N, layout=LAYOUTS[lay] if isinstance(lay, str) else int(lay),
                                       subset_size=int(pr.get("subset_size", N if self.mode == PNS_MODE_RF else 0)),
                                       num_chains=c, L0=int(pr.get("L0", 0)), betas=b.ctypes.data,
                                       beta=float(b[0])))
        o = pns_opts_default()
        o.dtype = dtype
        o.num_chains = 1
        o.L0 = L0
        o.seed = seed
        o.chain_id_base = chain_id_base
        o.init = INITS[init] if isinstance(init, str) else int(init)
        if x0 is not None:
            o.init = PNS_INIT_GIVEN
            self._x0 = np.ascontiguousarray(np.asarray(x0, dtype=np.uint8).ravel())
            o.x0 = self._x0.ctypes.data
        o.launch = LAUNCHES[launch] if isinstance(launch, str) else int(launch)
        o.chunk = chunk
        if stream is not None:
            o.stream = stream if isinstance(stream, int) else stream.cuda_stream
        o.log_capacity = log_capacity
        o.snapshot_every = snapshot_every
        o.snapshot_capacity = snapshot_capacity
        o.autotune = 1 if autotune else 0
        self.log_capacity = log_capacity
        self.snapshot_capacity = snapshot_capacity
        self.ctx = pns_create_batch(structs, self.mode, o)
        self.num_problems = pns_num_problems(self.ctx)
        self.info = [pns_problem_info_get(self.ctx, p) for p in range(self.num_problems)]
        self.num_chains = sum(i.num_chains for i in self.info)
        self.offsets = pns_chain_offsets(self.ctx, self.num_chains)

    def run(self, steps: int) -> "BatchSampler":
        pns_run(self.ctx, steps)
        return self

    def sync(self) -> None:
        pns_sync(self.ctx)

    def save(self) -> np.ndarray:
        """Checkpoint of every chain's state (pns_save) as a byte array."""
        buf = np.zeros(pns_save(self.ctx), np.uint8)
        pns_save(self.ctx, buf)
        return buf

    def load(self, buf) -> "BatchSampler":
        """Restore a checkpoint of an identically created batch (pns_load)."""
        b = np.ascontiguousarray(buf, dtype=np.uint8)
        pns_load(self.ctx, b, b.nbytes)
        return self

    def _split_bits(self, flat, rows: Optional[int] = None):
        out = []
        r = rows or 1
        for i in self.info:
            c0, c1 = i.chain_begin, i.chain_begin + i.num_chains
            seg = flat[self.offsets[c0] * r:self.offsets[c1] * r]
            out.append(seg.reshape(i.num_chains, r, i.N) if rows else seg.reshape(i.num_chains, i.N))
        return out

    def _split_chains(self, arr):
        return [arr[i.chain_begin:i.chain_begin + i.num_chains] for i in self.info]

    def read(self):
        s = np.zeros(self.offsets[-1], np.uint8)
        m = np.zeros(self.num_chains, np.int64)
        e = np.zeros(self.num_chains, np.float64)
        pns_read(self.ctx, s, m, e)
        return self._split_bits(s), self._split_chains(m), self._split_chains(e)

    def read_current(self):
        C = self.num_chains
        s = np.zeros(self.offsets[-1], np.uint8)
        e = np.zeros(C, np.float64)
        h = np.zeros(self.offsets[-1], _FIELD_DTYPES[pns_field_type(self.ctx)])
        L = np.zeros(C, np.int64)
        sub = np.zeros(C, np.int64)
        k = np.zeros(C, np.int64)
        pns_read_current(self.ctx, s, e, h, L, sub, k)
        return {"x": self._split_bits(s), "E": self._split_chains(e), "h": self._split_bits(h),
                "L": self._split_chains(L), "sub": self._split_chains(sub), "step": self._split_chains(k)}

    def read_log(self):
        C, K = self.num_chains, self.log_capacity
        a = np.zeros((C, K), np.int32)
        m = np.zeros((C, K), np.int64)
        e = np.zeros((C, K), np.float64)
        p = np.zeros((C, K), np.float64)
        pns_read_log(self.ctx, a, m, e, p)
        return {"action": self._split_chains(a), "M": self._split_chains(m), "E": self._split_chains(e),
                "p": self._split_chains(p)}

    def read_snapshots(self):
        C, S = self.num_chains, self.snapshot_capacity
        x = np.zeros(self.offsets[-1] * S, np.uint8)
        m = np.zeros((C, S), np.int64)
        e = np.zeros((C, S), np.float64)
        cnt = pns_read_snapshots(self.ctx, x, m, e)
        return self._split_bits(x, S), self._split_chains(m), self._split_chains(e), cnt

    def stats(self):
        arr = pns_stats(self.ctx, self.num_chains)
        return {k: np.array([getattr(s, k) for s in arr]) for k in ("steps", "flips", "stays", "saturated", "sum_M", "anomalies")}

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            pns_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ContSampler:
    """Unbiased PNS for continuous states (Alg 7) on the donut target of
    Sec 7, ``num_chains`` chains on the device (pns_cont_*)."""

    def __init__(self, num_chains: int = 1, *, dim: int = 2, pairs: int = 25, mu0: float = 9.0, sigma: float = 0.1,
                 L0: int = 1000, seed: int = 0, x0=None, chain_id_base: int = 0, log_capacity: int = 0, stream=None):
        o = pns_cont_opts()
        lib.pns_cont_opts_default(ctypes.byref(o))
        o.dim, o.pairs, o.mu0, o.sigma, o.L0, o.seed = dim, pairs, mu0, sigma, L0, seed
        o.num_chains, o.chain_id_base, o.log_capacity = num_chains, chain_id_base, log_capacity
        if x0 is not None:
            if hasattr(x0, "data_ptr"):
                self._x0 = x0.contiguous()
            else:
                self._x0 = np.ascontiguousarray(np.broadcast_to(np.asarray(x0, np.float64), (num_chains, dim)))
            o.x0 = _addr(self._x0)
        if stream is not None:
            o.stream = stream if isinstance(stream, int) else stream.cuda_stream
        self.num_chains, self.dim, self.pairs, self.log_capacity = num_chains, dim, pairs, log_capacity
        self.ctx = ctypes.c_void_p()
        _check(lib.pns_cont_create(ctypes.byref(self.ctx), ctypes.byref(o)))

    def run(self, steps: int) -> "ContSampler":
        _check(lib.pns_cont_run(self.ctx, steps))
        return self

    def sync(self) -> None:
        _check(lib.pns_cont_sync(self.ctx))

    def read(self):
        C, d = self.num_chains, self.dim
        x = np.zeros((C, d))
        lp = np.zeros(C)
        L = np.zeros(C, np.int64)
        st = np.zeros(C, np.int64)
        k = np.zeros(C, np.int64)
        _check(lib.pns_cont_read(self.ctx, x.ctypes.data, lp.ctypes.data, L.ctypes.data, st.ctypes.data,
                                 k.ctypes.data))
        return {"x": x, "lp": lp, "L": L, "set": st, "step": k}

    def read_log(self):
        C, K = self.num_chains, self.log_capacity
        a = np.zeros((C, K), np.int32)
        m = np.zeros((C, K), np.int64)
        lp = np.zeros((C, K))
        p = np.zeros((C, K))
        w = np.zeros((C, K))
        _check(lib.pns_cont_read_log(self.ctx, a.ctypes.data, m.ctypes.data, lp.ctypes.data, p.ctypes.data,
                                     w.ctypes.data))
        return {"action": a, "M": m, "E": lp, "p": p, "w": w}

    def read_sums(self):
        out = np.zeros((self.num_chains, 2, 4 * self.dim + 1))
        _check(lib.pns_cont_read_sums(self.ctx, out.ctypes.data))
        return out

    def clear_sums(self) -> "ContSampler":
        _check(lib.pns_cont_clear_sums(self.ctx))
        return self

    def stats(self):
        j = np.zeros(self.num_chains, np.int64)
        s = np.zeros(self.num_chains, np.int64)
        _check(lib.pns_cont_stats(self.ctx, j.ctypes.data, s.ctypes.data))
        return {"jumps": j, "stays": s}

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib.pns_cont_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
