"""Throughput benchmark of the PNS sampler on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workload (default ``rf_n1024_int16``): Rejection-Free on a dense symmetric
int16 QUBO, N = 1024, entries uniform on {-100..100}, 1024 chains,
beta = 0.01, int32 local fields.  One benchmark step runs every chain for
``--chain-steps`` sampler steps (default 100000, the full per-chain length of
the workload) in the persistent launch form, with all inputs resident in HBM.
The JSON line reports flips/s (value) and effective Metropolis steps/s
(sum of multiplicities per second), the HBM roofline of the dominant kernel
(bytes of Q read per flip = N * sizeof(int16)), the VALU issue roofline of
the same kernel (wave64 VALU instructions per chain step from its counter
run), the same workload with Basic
PNS subset 64 and in the plain one-launch-per-step form, and the CPU oracle
timed on a bounded sample on this host.

Other workloads (--workload): basic64_n1024_int16, unbiased_n8192_f32
(Unbiased PNS, N = 8192 float32, 4096 chains), batched64_uneven_int16 (64
problems of uneven N in one context), fit_n64_f32 / fit_n512_f32
(maximum-likelihood fit through the MFMA moment kernel), donut_cont_f64
(continuous Unbiased PNS, Alg 7, on the donut target of Sec 6).
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


def _measured_traffic(workload: str, chain_steps: int):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter runs (profiles/hbm_traffic.txt), or None when no run matches the
    workload and launch length or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    src = os.path.join(ROOT, "paper_2210_10513_amd", "csrc", "pns_step.h")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        f = line.split()
        if len(f) == 6 and not line.startswith("#") and f[0] == workload and int(f[1]) == chain_steps and f[2] == sha:
            return float(f[5])
    return None


# Wave64 VALU issue peak: 256 CUs x 4 SIMDs, each SIMD16 issuing one wave64
# instruction per 4 cycles, at 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def _valu_per_chain_step(workload: str, tile):
    """VALU instructions (wave64) per chain step of the step kernel from the
    committed SQ counter runs (profiles/valu_issue.txt), or None when no run
    matches the workload and tile (block, groups) or the kernel source changed
    since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "valu_issue.txt")
    src = os.path.join(ROOT, "paper_2210_10513_amd", "csrc", "pns_step.h")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        f = line.split()
        if (len(f) == 6 and not line.startswith("#") and f[0] == workload and f[1] == "%dx%d" % tuple(tile)
                and f[2] == sha):
            return float(f[3]) / float(f[4])
    return None


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
    if name == "donut_cont_f64":
        return dict(cont=True, dim=2, pairs=25, mu0=9.0, sigma=0.1, L0=1000, chains=65536, steps=4000,
                    desc="donut_d2_mu9_sigma0.1_pairs25_L1000_65536chains")
    if name in ("fit_n64_f32", "fit_n512_f32"):
        N = 64 if name == "fit_n64_f32" else 512
        w = inputs.c5_fit(N)
        return dict(fit=True, Q=w.Q, betas=w.betas, mode="rf", n=0, L0=100, qbytes=4, steps=0, desc=w.name)
    raise SystemExit(f"unknown workload {name}")


def _bench_fit(args, wl):
    """Maximum-likelihood fit of a QUBO to 2^20 weighted samples of a seeded
    ground truth (8192 chains, burn-in 8N steps, 128 snapshots 16 steps
    apart).  One bench step is one gradient iteration of fit_qubo: the
    warm-started sampler runs 8192 chains for 64 + 16 x 8 steps, the backward
    pass runs the bf16 MFMA moment kernel on the 131072 snapshot records, and
    the centered momentum update follows.  Also reported: the backward kernel
    timed alone, and the quality of a 300-iteration fit (moment gap against
    the sampling-noise floor of the true Q, relative parameter error)."""
    import torch
    from paper_2210_10513_amd import binding
    from paper_2210_10513_amd.autograd import ChainOptions, LogZ, fit_qubo, moments_of_samples, release
    dev = torch.device("cuda")
    N = wl["Q"].shape[0]
    beta = 1.0
    Qt = torch.tensor(wl["Q"], device=dev)
    D, nsamp = moments_of_samples(Qt, beta, ChainOptions(num_chains=8192, burn_in=8 * N, samples=128, every=16,
                                                         seed=1))
    chains, burn, samples, every, lr = 8192, 64, 16, 8, 0.1
    state = {}
    opts = ChainOptions(num_chains=chains, burn_in=burn, samples=samples, every=every, seed=3, state=state,
                        exact_max=0)
    res = fit_qubo(D, beta, max(1, args.warmup), lr, opts)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    res = fit_qubo(D, beta, args.steps, lr, opts, Q0=res.Q)
    t1.record(stream)
    torch.cuda.synchronize()
    sec = t0.elapsed_time(t1) / 1000.0 / args.steps
    steps_per_iter = burn + samples * every
    flips = chains * steps_per_iter  # Rejection-Free: every record is a flip
    # fit quality over 300 iterations from zero, and the noise floor: the
    # gap of the true Q's own sampled moments (long burn-in) to the data's
    q = fit_qubo(D, beta, 300, lr, opts)
    rel = float((q.Q - Qt).norm() / Qt.norm())
    Qg = Qt.clone().requires_grad_(True)
    LogZ.apply(Qg, beta, ChainOptions(num_chains=chains, burn_in=8 * N, samples=samples, every=every, seed=5,
                                      exact_max=0)).backward()
    floor = float((D.float() + Qg.grad / beta).abs().max())

    # backward kernel alone: the moments of one iteration's snapshots
    s = state["sampler"]
    G = torch.empty((N, N), dtype=torch.float64, device=dev)
    sm = torch.empty(1, dtype=torch.float64, device=dev)
    for _ in range(3):
        binding.pns_snapshot_moments(s.ctx, 0, G, sum_m=sm)
    reps = 50
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        binding.pns_snapshot_moments(s.ctx, 0, G, sum_m=sm)
    e1.record(stream)
    torch.cuda.synchronize()
    release(state)
    mom_ms = e0.elapsed_time(e1) / reps
    K = chains * samples
    mflops = 2.0 * K * N * N
    mom_tf = mflops / (mom_ms * 1e-3) / 1e12
    out = {
        "metric": "flips/s", "value": flips / sec, "unit": "flips/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1000.0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "N": N, "chains": chains, "mode": "rf", "beta": beta,
                   "data_samples": int(nsamp), "records_per_gradient": K, "steps_per_gradient": steps_per_iter,
                   "lr": lr, "update": "centered momentum 0.9"},
        "gradients_per_s": 1.0 / sec,
        "fit_300": {"moment_gap_mean_last50": float(np.mean(q.moment_gap[-50:])), "noise_floor": floor,
                    "rel_param_error": rel},
        "roofline": {"bound": "hbm", "achieved": flips * N * 4 / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": flips * N * 4 / sec / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_flip": N * 4, "kernel": "step_kernel + moments (whole iteration)",
                     "kernel_avg_ms": sec * 1000.0},
        "moments_roofline": {"bound": "mfma", "achieved": mom_tf, "peak": 2500.0, "unit": "TFLOP/s",
                             "frac": mom_tf / 2500.0, "traffic": None, "flops_per_launch": mflops,
                             "kernel": "moments (fill + prep + pack + moments_kernel + reduce + sum)",
                             "kernel_avg_ms": mom_ms},
    }
    print(json.dumps(out))


# FP64 operations per neighbour evaluation of the continuous sampler: y = x + s
# (D adds), |y|^2 (D multiplies, D adds), (|y|^2 - mu0)^2 / (2 sigma^2) (3),
# the log-density difference (1), min(0, .) (1), and exp counted as 20 (range
# reduction, a degree-11 polynomial, scaling).
def _cont_flops_per_neighbour(D: int) -> int:
    return 4 * D + 5 + 20


FP64_VECTOR_PEAK_TFLOPS = 78.6


def _bench_cont(args, wl):
    """Continuous Unbiased PNS (Alg 7) on the donut target of Sec 6: d = 2,
    mu0 = 9, sigma = 0.1, 25 pairs (50 neighbours), L0 = 1000; 65536 chains
    from exact draws of the target.  One bench step runs every chain for
    --chain-steps records (default 4000).  Value: original (Metropolis-
    equivalent) samples per second, the unit of the Sec 6 comparison."""
    import torch
    from paper_2210_10513_amd import inputs
    from paper_2210_10513_amd.binding import ContSampler
    chain_steps = args.chain_steps or wl["steps"]
    C, d = wl["chains"], wl["dim"]
    x0 = inputs.donut_draws(C, d, wl["mu0"], wl["sigma"], seed=1)
    stream = torch.cuda.current_stream()
    s = ContSampler(C, dim=d, pairs=wl["pairs"], mu0=wl["mu0"], sigma=wl["sigma"], L0=wl["L0"], seed=2, x0=x0,
                    stream=stream)
    for _ in range(args.warmup):
        s.run(chain_steps)
    s.sync()
    S0 = s.read_sums()[:, 0, 0].sum()
    st0 = s.stats()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        s.run(chain_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1000.0 / args.steps
    S1 = s.read_sums()[:, 0, 0].sum()
    st1 = s.stats()
    s.close()
    orig = (S1 - S0) / args.steps
    recs = float(C) * chain_steps
    jumps = float((st1["jumps"] - st0["jumps"]).sum()) / args.steps
    nbr = recs * 2 * wl["pairs"]
    flops = nbr * _cont_flops_per_neighbour(d)
    launches = -(-chain_steps // 8192)
    achieved = flops / sec / 1e12
    out = {
        "metric": "original_samples/s", "value": orig / sec, "unit": "original samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1000.0, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "dim": d, "pairs": wl["pairs"], "mu0": wl["mu0"], "sigma": wl["sigma"],
                   "L0": wl["L0"], "chains": C, "records_per_chain_per_step": chain_steps},
        "records_per_s": recs / sec, "jumps_per_s": jumps / sec, "neighbour_evaluations_per_s": nbr / sec,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_neighbour": _cont_flops_per_neighbour(d), "kernel": "cont_kernel",
                     "kernel_avg_ms": sec * 1000.0 / launches},
    }
    if not args.no_cpu:
        import oracle
        K = 200
        t0 = time.perf_counter()
        oracle.cont_run(x0[:8], K, mu0=wl["mu0"], sigma=wl["sigma"], pairs=wl["pairs"], L0=wl["L0"], seed=2,
                        log=False)
        dt = time.perf_counter() - t0
        K = max(200, int(K * 12.0 / max(dt, 1e-6)))
        t0 = time.perf_counter()
        r = oracle.cont_run(x0[:8], K, mu0=wl["mu0"], sigma=wl["sigma"], pairs=wl["pairs"], L0=wl["L0"], seed=2,
                            log=False)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": float(r.sums[:, 0, 0].sum()) / dt, "unit": "original samples/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"8 chains x {K} records of the same workload, single-threaded FP64 oracle "
                                         f"({dt:.1f} s)"}
    print(json.dumps(out))


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


def _cpu_baseline(wl, budget_s: float = 15.0):
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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer 3 times (reference for the HBM byte counters)")
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
    if args.copy_calibration:
        # 2^28 float32 = 1 GiB read and 1 GiB written per copy: the scale of
        # the FETCH_SIZE / WRITE_SIZE counters for a kernel of known traffic
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "copies": 3}))
        return

    wl = _workload(args.workload)
    if wl.get("cont"):
        _bench_cont(args, wl)
        return
    if wl.get("fit"):
        _bench_fit(args, wl)
        return
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
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _measured_traffic(args.workload, chain_steps) if args.steps >= 1 else None,
                     "bytes_per_flip": bytes_per_flip, "kernel": "step_kernel",
                     "kernel_avg_ms": sec * 1000.0},
    }
    vps = _valu_per_chain_step(args.workload, tile)
    if vps is not None:
        # the bound of an L2-resident step: wave64 VALU issue (records = loop iterations)
        out["issue_roofline"] = {"bound": "alu", "achieved": vps * recs / sec, "peak": VALU_ISSUE_PEAK,
                                 "unit": "wave64 VALU instr/s", "frac": vps * recs / sec / VALU_ISSUE_PEAK,
                                 "valu_per_chain_step": vps}
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
