"""Throughput benchmark of the PNS sampler on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workload (default ``rf_n1024_int16``): Rejection-Free on a dense symmetric
int16 QUBO, N = 1024, entries uniform on {-100..100}, 1024 chains,
beta = 0.01, int32 local fields.  One benchmark step runs every chain for
``--chain-steps`` sampler steps (default 100000, the full per-chain length of
the workload) in the persistent launch form, with all inputs resident in HBM.
The JSON line reports flips/s (value) and effective Metropolis steps/s
(sum of multiplicities per second), the HBM roofline of the dominant kernel
(bytes of Q read per flip = N * sizeof(int16)), the same workload with Basic
PNS subset 64 and in the plain one-launch-per-step form, and the CPU oracle
timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _workload(name: str):
    from paper_2210_10513_amd import inputs
    if name == "rf_n1024_int16":
        w = inputs.c2_rf_n1024(mode="rf")
        return dict(Q=w.Q, betas=w.betas, mode="rf", n=0, L0=100, qbytes=2, steps=w.steps, desc=w.name)
    if name == "basic64_n1024_int16":
        w = inputs.c2_rf_n1024(mode="basic")
        return dict(Q=w.Q, betas=w.betas, mode="basic", n=64, L0=100, qbytes=2, steps=w.steps, desc=w.name)
    if name == "unbiased_n8192_f32":
        w = inputs.c3_unbiased_n8192()
        return dict(Q=w.Q, betas=w.betas, mode="unbiased_sys", n=512, L0=100, qbytes=4, steps=w.steps, desc=w.name)
    if name == "batched64_uneven_int16":
        w = inputs.c4_batched()
        cp = int(w.extra["chains_per"])
        probs = [{"Q": Q, "num_chains": cp, "beta": w.betas[i * cp:(i + 1) * cp], "subset_size": 0}
                 for i, Q in enumerate(w.Q)]
        return dict(problems=probs, betas=w.betas, mode="unbiased_sys", n=0, L0=100, qbytes=2, steps=20_000,
                    desc=w.name, Ns=np.asarray(w.extra["Ns"]))
    raise SystemExit(f"unknown workload {name}")


def _time_batch(wl, chain_steps: int, steps: int, warmup: int, launch: str, seed: int):
    """Batched context over every problem of the workload (subset sizes and
    tiles from the autotuner).  Returns (seconds per bench step, flips, Q
    bytes streamed, records, sum M per bench step, problem infos)."""
    import torch
    from paper_2210_10513_amd.binding import BatchSampler
    stream = torch.cuda.current_stream()
    s = BatchSampler(wl["problems"], wl["mode"], L0=wl["L0"], seed=seed, launch=launch, stream=stream)
    nbits = np.concatenate([np.full(i.num_chains, i.N) for i in s.info]).astype(np.float64)
    for _ in range(warmup):
        s.run(chain_steps)
    s.sync()
    st0 = s.stats()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    for _ in range(steps):
        s.run(chain_steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    st1 = s.stats()
    info = [(i.N, i.subset_size, i.block, i.groups, i.flavour) for i in s.info]
    s.close()
    dflips = (st1["flips"] - st0["flips"]).astype(np.float64)
    flips = float(dflips.sum()) / steps
    qbytes = float((dflips * nbits).sum()) * wl["qbytes"] / steps
    recs = float((st1["steps"] - st0["steps"]).sum()) / steps
    summ = float((st1["sum_M"] - st0["sum_M"]).sum()) / steps
    return ms / 1000.0 / steps, flips, qbytes, recs, summ, info


def _bench_batch(args, wl):
    chain_steps = args.chain_steps or wl["steps"]
    launch = args.launch if args.launch != "persistent" else "graph"
    t0 = time.perf_counter()
    sec, flips, qb, recs, summ, info = _time_batch(wl, chain_steps, args.steps, args.warmup, launch, seed=1)
    setup = time.perf_counter() - t0
    achieved = qb / sec / 1e9
    out = {
        "metric": "flips/s", "value": flips / sec, "unit": "flips/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1000.0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": wl["desc"], "problems": len(info), "chains": int(len(wl["betas"])),
                   "N_min": int(min(i[0] for i in info)), "N_max": int(max(i[0] for i in info)),
                   "mode": wl["mode"], "subset": "autotuned", "chain_steps_per_step": chain_steps, "launch": launch,
                   "subset_sizes": [int(i[1]) for i in info], "tiles": sorted({f"{i[2]}x{i[3]}" for i in info})},
        "effective_mh_steps_per_s": summ / sec,
        "records_per_s": recs / sec,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_flip": "N_p * 2 for the flipping chain's problem", "kernel": "step_kernel (all classes)",
                     "kernel_avg_ms": sec * 1000.0},
        "setup_s": setup,
    }
    if not args.no_extras:
        sp, fp, qp, _, _, _ = _time_batch(wl, 100, 1, 1, "plain", seed=3)
        out["variants"] = {"plain_launch_flips_per_s": fp / sp, "batched_over_plain": (flips / sec) / (fp / sp)}
    print(json.dumps(out))


def _time_sampler(wl, chain_steps: int, steps: int, warmup: int, launch: str, seed: int, tile=(0, 0)):
    """Returns (seconds per bench step, flips per bench step, sum M per bench step)."""
    import torch
    from paper_2210_10513_amd.binding import Sampler
    stream = torch.cuda.current_stream()
    s = Sampler(wl["Q"], wl["betas"], wl["n"], wl["mode"], num_chains=len(wl["betas"]), L0=wl["L0"], seed=seed,
                launch=launch, stream=stream, block=tile[0], groups=tile[1])
    for _ in range(warmup):
        s.run(chain_steps)
    s.sync()
    st0 = s.stats()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t_start.record(stream)
    for _ in range(steps):
        s.run(chain_steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t_start.elapsed_time(t_end)
    st1 = s.stats()
    tile = s.tile()
    s.close()
    flips = float((st1["flips"] - st0["flips"]).sum()) / steps
    recs = float((st1["steps"] - st0["steps"]).sum()) / steps
    summ = float((st1["sum_M"] - st0["sum_M"]).sum()) / steps
    return ms / 1000.0 / steps, flips, recs, summ, wall, tile


def _cpu_baseline(wl, budget_s: float = 12.0):
    import oracle
    Q = wl["Q"].astype(np.int64) if np.issubdtype(wl["Q"].dtype, np.integer) else wl["Q"].astype(np.float64)
    modes = {"rf": oracle.MODE_RF, "basic": oracle.MODE_BASIC, "unbiased_sys": oracle.MODE_UNBIASED_SYS}
    chains = 4
    # calibrate on a short run, then size the sample to the budget
    K = 200
    t0 = time.perf_counter()
    oracle.run(Q, wl["betas"][:chains], modes[wl["mode"]], K, n=wl["n"], L0=wl["L0"], seed=1, num_chains=chains,
               log=False)
    dt = time.perf_counter() - t0
    K = max(200, int(K * budget_s / max(dt, 1e-6)))
    t0 = time.perf_counter()
    r = oracle.run(Q, wl["betas"][:chains], modes[wl["mode"]], K, n=wl["n"], L0=wl["L0"], seed=1,
                   num_chains=chains, log=False)
    dt = time.perf_counter() - t0
    flips = float(r.flips.sum())
    return {"value": flips / dt, "unit": "flips/s", "cores": 1, "kind": "oracle",
            "sample": f"{chains} chains x {K} steps of the same workload, single-threaded FP64/int64 oracle "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rf_n1024_int16")
    ap.add_argument("--chain-steps", type=int, default=0, help="sampler steps per chain per bench step (0 = workload)")
    ap.add_argument("--launch", default="persistent")
    ap.add_argument("--tile", default="", help="workgroup size and 4-field groups per lane, e.g. 64,4")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: chains are independent, so nothing here runs on more than one "
              "(see the sharding note in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)

    wl = _workload(args.workload)
    if "problems" in wl:
        _bench_batch(args, wl)
        return
    chain_steps = args.chain_steps or wl["steps"]
    C = len(wl["betas"])
    N = wl["Q"].shape[0]
    tile_req = tuple(int(v) for v in args.tile.split(",")) if args.tile else (0, 0)
    sec, flips, recs, summ, wall, tile = _time_sampler(wl, chain_steps, args.steps, args.warmup, args.launch, seed=1,
                                                       tile=tile_req)
    value = flips / sec
    bytes_per_flip = N * wl["qbytes"]
    achieved = flips * bytes_per_flip / sec / 1e9
    out = {
        "metric": "flips/s",
        "value": value,
        "unit": "flips/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if wl["qbytes"] == 2 else "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "N": N, "chains": C, "mode": wl["mode"], "subset": wl["n"] or N,
                   "beta": float(wl["betas"][0]), "chain_steps_per_step": chain_steps, "launch": args.launch,
                   "tile": list(tile)},
        "effective_mh_steps_per_s": summ / sec,
        "records_per_s": recs / sec,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_flip": bytes_per_flip, "kernel": "step_kernel",
                     "kernel_avg_ms": sec * 1000.0},
    }
    if not args.no_extras and args.workload == "rf_n1024_int16":
        extras = {}
        wb = _workload("basic64_n1024_int16")
        s2, f2, r2, m2, _, t2 = _time_sampler(wb, chain_steps // 4, 1, 1, "persistent", seed=2)
        extras["basic64_flips_per_s"] = f2 / s2
        extras["basic64_effective_mh_steps_per_s"] = m2 / s2
        sp, fp, rp, mp, _, _ = _time_sampler(wl, 200, 1, 1, "plain", seed=3)
        extras["plain_launch_flips_per_s"] = fp / sp
        extras["persistent_over_plain"] = value / (fp / sp)
        out["variants"] = extras
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
