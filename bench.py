"""Throughput benchmark of the PNS sampler on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload (``batched64_uneven_int16``): Unbiased PNS with systematic
partial neighbor sets over 64 dense-stored int16 QUBOs of uneven size (N
log-uniform in [256, 16384], half the entries zero, entries uniform on
{-100..100}), 64 chains each (4096 chains), beta = 0.01 sqrt(2048 / N),
subset sizes and tiles from the autotuner, in one context whose launch
classes run concurrently, captured in a HIP graph.  One benchmark step runs
every chain for ``--chain-steps`` sampler steps (default 100000, the full
per-chain length), with all inputs resident in HBM.  The JSON line reports
aggregate flips/s (value), effective Metropolis steps/s (sum of
multiplicities per second), the HBM roofline of the dominant kernel (the
launch class on the critical path: bytes of Q read per flip = N * 2 over its
kernel time, from HIP events on that class's stream), the same for the
problems with N >= 8192, every class's figures, the batched form against
the plain one-launch-per-step form, the Unbiased PNS N = 8192 float32 and
Rejection-Free N = 1024 int16 workloads as extra keys, and the CPU oracle
timed on a bounded sample of the workload on one core and on every core.

Other workloads (--workload): rf_n1024_int16, basic64_n1024_int16,
unbiased_n8192_f32 (single-problem contexts), fit_n64_f32 / fit_n512_f32
(maximum-likelihood fit through the MFMA moment kernel), donut_cont_f64
(continuous Unbiased PNS, Alg 7, on the donut target of Sec 7).
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

# Hardware queues of this process (--hw-queues, default 12, or 8 with
# --launch graph; read when HIP starts, so taken from the command line before
# anything touches the GPU):
# the batched workload's launch classes, eight, run on one stream each next
# to the context's own stream, and each stream needs a queue of its own so
# that all classes run at once.  Measured on one MI355X, ms per step of the
# batch with its launches queued directly on the streams: 664-666 at 12
# queues, 667-676 at 10, 794-816 at 9 and 770-805 at 8 (two classes share a
# queue and run one after the other); replaying the captured graph instead,
# which maps its branches onto queues itself: 670-705 at 8, 688-694 at 9,
# 688-788 at 10, 846-861 at 12, 833-870 at HIP's default of 4.


def _hw_queues_arg() -> str:
    graph = False
    for i, a in enumerate(sys.argv):
        if a == "--hw-queues" and i + 1 < len(sys.argv):
            return sys.argv[i + 1]
        if a.startswith("--hw-queues="):
            return a.split("=", 1)[1]
        if (a == "--launch" and i + 1 < len(sys.argv) and sys.argv[i + 1] == "graph") or a == "--launch=graph":
            graph = True
    return "8" if graph else "12"


os.environ["GPU_MAX_HW_QUEUES"] = _hw_queues_arg()

HBM_PEAK_GBS = 8000.0


def _kernel_sha(window: bool = False) -> str:
    """sha256 prefix of a sampling kernel's sources: the step kernel's
    (pns_step.h), or the window kernel's (pns_step.h, then pns_wave.h, which
    includes it).  A committed counter row applies while it is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for name in ("pns_step.h", "pns_wave.h") if window else ("pns_step.h",):
        h.update(open(os.path.join(ROOT, "paper_2210_10513_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def _measured_traffic(workload: str, chain_steps: int, window: bool = False):
    """HBM bytes per launch of the step kernel (window: the window kernel)
    from the committed rocprofv3 counter runs (profiles/hbm_traffic.txt), or
    None when no run matches the workload and launch length or the kernel's
    sources changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    sha = _kernel_sha(window)
    for line in open(path):
        f = line.split()
        if len(f) == 6 and not line.startswith("#") and f[0] == workload and int(f[1]) == chain_steps and f[2] == sha:
            return float(f[5])
    return None


# Wave64 VALU issue peak: 256 CUs x 4 SIMDs, each SIMD16 issuing one wave64
# instruction per 4 cycles, at 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def _valu_per_chain_step(workload: str, tile, window: bool = False):
    """VALU instructions (wave64) per chain step of the step kernel (window:
    the window kernel) from the committed SQ counter runs
    (profiles/valu_issue.txt), or None when no run matches the workload and
    tile (block, groups) or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "valu_issue.txt")
    if not os.path.exists(path):
        return None
    sha = _kernel_sha(window)
    for line in open(path):
        f = line.split()
        if (len(f) == 6 and not line.startswith("#") and f[0] == workload and f[1] == "%dx%d" % tuple(tile)
                and f[2] == sha):
            return float(f[3]) / float(f[4])
    return None


def _batch_issue_roofline(classes, chain_steps: int, sec_per_step: float):
    """Wave64 VALU issue of the whole batch: every class's VALU instructions
    per chain step (committed SQ counter runs) times its chain steps, over the
    step time, against the issue peak; None unless every class has a row for
    its current kernel source."""
    total = 0.0
    for c in classes:
        b, g = (int(v) for v in c["tile"].split("x"))
        vps = _valu_per_chain_step(_class_key(c), (b, g), c["flavour"] == 5)
        if vps is None:
            return None
        total += vps * c["chains"] * chain_steps
    achieved = total / sec_per_step
    return {"bound": "alu", "achieved": achieved, "peak": VALU_ISSUE_PEAK, "unit": "wave64 VALU instr/s",
            "frac": achieved / VALU_ISSUE_PEAK, "valu_per_step": total,
            "scope": "every launch class's VALU instructions per chain step (SQ counters) x its chain steps, "
                     "over the step time"}


def _class_key(c) -> str:
    """Counter-table key of a launch class of the batched workload: its tile,
    kernel flavour and chains (the autotuner's choices, which a run may make
    differently, decide which problems form a class)."""
    return f"batched64_class_{c['tile']}_f{c['flavour']}_c{c['chains']}_N{c['N_min']}-{c['N_max']}"


def _kernel_name(c) -> str:
    """Kernel of a launch class of 16-bit coefficients with 32-bit fields."""
    block, groups = (int(v) for v in c["tile"].split("x"))
    if c["flavour"] == 5:
        return f"wave_kernel<short, {block // 64}, {groups}, false>"
    return f"step_kernel<short, int, {block}, {groups}, {c['flavour']}, false>"


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
        return dict(problems=probs, betas=w.betas, mode="unbiased_sys", n=0, L0=100, qbytes=2, steps=w.steps,
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
    """Continuous Unbiased PNS (Alg 7) on the donut target of Sec 7: d = 2,
    mu0 = 9, sigma = 0.1, 25 pairs (50 neighbours), L0 = 1000; 65536 chains
    from exact draws of the target.  One bench step runs every chain for
    --chain-steps records (default 4000).  Value: original (Metropolis-
    equivalent) samples per second, the unit of the Sec 7 comparison."""
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


def _class_rows(prof, sec_scale: float):
    """Per-class figures from pns_profile_read: kernel time per launch, flips/s
    and GB/s of algorithmic row bytes over that kernel time."""
    rows = []
    for k in prof:
        ms = k["kernel_ms"] / max(1, k["launches"])
        gbs = k["row_bytes"] / max(k["kernel_ms"], 1e-12) / 1e6
        rows.append({"tile": f"{k['block']}x{k['groups']}", "flavour": k["flavour"], "chains": k["chains"],
                     "N_min": k["N_min"], "N_max": k["N_max"], "launches": k["launches"],
                     "kernel_avg_ms": ms, "flips_per_launch": k["flips"] / max(1, k["launches"]),
                     "bytes_per_launch": k["row_bytes"] / max(1, k["launches"]),
                     "flips_per_s": k["flips"] / max(k["kernel_ms"] * 1e-3, 1e-12), "GB_per_s": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS})
    return rows


def _time_batch(wl, chain_steps: int, steps: int, warmup: int, launch: str, seed: int, profile: bool = True):
    """Batched context over every problem of the workload (subset sizes and
    tiles from the autotuner).  The K timed steps in the requested launch
    form are bracketed by HIP events on the context's stream.  With
    `profile`, K further steps run with per-class timing (pns_profile: HIP
    events on each launch class's own stream; a graph context queues the
    same launches directly while profiling).  Returns a dict of figures."""
    import torch
    from paper_2210_10513_amd import binding as bd
    from paper_2210_10513_amd.binding import BatchSampler
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    s = BatchSampler(wl["problems"], wl["mode"], L0=wl["L0"], seed=seed, launch=launch, stream=stream)
    setup = time.perf_counter() - t0
    C = s.num_chains
    nbits = np.concatenate([np.full(i.num_chains, i.N) for i in s.info]).astype(np.float64)

    def timed():
        st0 = s.stats()
        torch.cuda.synchronize()
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        t_start.record(stream)
        for _ in range(steps):
            s.run(chain_steps)
        t_end.record(stream)
        torch.cuda.synchronize()
        st1 = s.stats()
        d = {k: (st1[k] - st0[k]).astype(np.float64) / steps for k in ("flips", "steps", "sum_M")}
        return t_start.elapsed_time(t_end) / 1000.0 / steps, d

    for _ in range(warmup):
        s.run(chain_steps)
    s.sync()
    sec, d = timed()
    out = {"sec": sec, "flips": float(d["flips"].sum()), "qbytes": float((d["flips"] * nbits).sum()) * wl["qbytes"],
           "records": float(d["steps"].sum()), "sum_M": float(d["sum_M"].sum()), "setup_s": setup,
           "info": [(i.N, i.subset_size, i.block, i.groups, i.flavour) for i in s.info], "chain_N": nbits,
           "chain_class": bd.pns_class_of_chain(s.ctx, C), "prof": None}
    if profile:
        bd.pns_profile(s.ctx, True)
        psec, pd = timed()
        out["prof"] = bd.pns_profile_read(s.ctx)
        bd.pns_profile(s.ctx, False)
        out["prof_sec"] = psec
        out["prof_dflips"] = pd["flips"]
    s.close()
    return out


def _bench_batch(args, wl, cpu_spec=None):
    chain_steps = args.chain_steps or wl["steps"]
    launch = args.launch
    r = _time_batch(wl, chain_steps, args.steps, args.warmup, launch, seed=1)
    sec, flips, info = r["sec"], r["flips"], r["info"]
    achieved_all = r["qbytes"] / sec / 1e9
    classes = _class_rows(r["prof"], 1.0)
    # the dominant kernel: the launch class with the longest kernel time (the
    # critical path of the concurrently running classes)
    dom = max(range(len(classes)), key=lambda i: classes[i]["kernel_avg_ms"])
    dk = classes[dom]
    # problems with N >= 8192: their flips' row bytes over the longest kernel
    # time among the classes that hold them (a lower bound on their own rate)
    big = r["chain_N"] >= 8192
    big_cls = sorted({int(c) for c in r["chain_class"][big]})
    big_ms = max(classes[i]["kernel_avg_ms"] for i in big_cls) if big_cls else 0.0
    big_bytes = float((r["prof_dflips"][big] * r["chain_N"][big]).sum()) * wl["qbytes"]
    big_gbs = big_bytes / (big_ms * 1e-3) / 1e9 if big_ms else 0.0
    out = {
        "metric": "flips/s", "value": flips / sec, "unit": "flips/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1000.0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": wl["desc"], "problems": len(info), "chains": int(len(wl["betas"])),
                   "N_min": int(min(i[0] for i in info)), "N_max": int(max(i[0] for i in info)),
                   "mode": wl["mode"], "subset": "autotuned", "chain_steps_per_step": chain_steps, "launch": launch,
                   "subset_sizes": [int(i[1]) for i in info], "tiles": sorted({f"{i[2]}x{i[3]}" for i in info}),
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "effective_mh_steps_per_s": r["sum_M"] / sec,
        "records_per_s": r["records"] / sec,
        "roofline": {"bound": "hbm", "achieved": dk["GB_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dk["hbm_frac"],
                     "traffic": _measured_traffic(_class_key(dk), chain_steps, dk["flavour"] == 5),
                     "bytes_per_flip": "N * 2 of the flipping chain's problem",
                     "kernel": f"{_kernel_name(dk)} "
                               f"(launch class N {dk['N_min']}..{dk['N_max']}, {dk['chains']} chains)",
                     "kernel_avg_ms": dk["kernel_avg_ms"], "bytes_per_launch": dk["bytes_per_launch"],
                     "timing": f"HIP events on the class's stream over {args.steps} further steps with the "
                               f"launches queued directly (step {r['prof_sec'] * 1e3:.1f} ms there, "
                               f"{sec * 1e3:.1f} ms in the timed {launch} form)"},
        "n_ge_8192": {"problems": int(sum(1 for i in info if i[0] >= 8192)), "chains": int(big.sum()),
                      "flips_per_s": float(r["prof_dflips"][big].sum()) / (big_ms * 1e-3) if big_ms else 0.0,
                      "GB_per_s": big_gbs, "hbm_frac": big_gbs / HBM_PEAK_GBS, "kernel_ms": big_ms,
                      "classes": [classes[i]["tile"] + "/f" + str(classes[i]["flavour"]) for i in big_cls]},
        "whole_batch": {"GB_per_s": achieved_all, "hbm_frac": achieved_all / HBM_PEAK_GBS,
                        "note": "all classes' row bytes over the step time (classes overlap)"},
        "classes": classes,
        "setup_s": r["setup_s"],
    }
    issue = _batch_issue_roofline(classes, chain_steps, sec)
    if issue is not None:
        out["issue_roofline"] = issue
    if not args.no_extras:
        # the N >= 8192 problems on their own (same chains, same kernels):
        # their rate when they do not share the GPU with the rest of the batch
        big_wl = dict(wl, problems=[pr for pr in wl["problems"] if pr["Q"].shape[0] >= 8192])
        b = _time_batch(big_wl, chain_steps, 1, 1, launch, seed=1)
        bcl = _class_rows(b["prof"], 1.0)
        out["n_ge_8192"]["alone"] = {
            "flips_per_s": b["flips"] / b["sec"], "GB_per_s": b["qbytes"] / b["sec"] / 1e9,
            "hbm_frac": b["qbytes"] / b["sec"] / 1e9 / HBM_PEAK_GBS, "ms_per_step": b["sec"] * 1e3,
            "classes": [{k: c[k] for k in ("tile", "flavour", "chains", "kernel_avg_ms", "GB_per_s", "hbm_frac")}
                        for c in bcl]}
        p = _time_batch(wl, 100, 1, 1, "plain", seed=3, profile=False)
        out["variants"] = {"plain_launch_flips_per_s": p["flips"] / p["sec"],
                           "batched_over_plain": (flips / sec) / (p["flips"] / p["sec"])}
        out["extra_workloads"] = {name: _single_summary(name, args) for name in
                                  ("unbiased_n8192_f32", "rf_n1024_int16")}
    if cpu_spec is not None:
        out["cpu_baseline"] = _cpu_baseline(dict(cpu_spec, subsets=[int(i[1]) for i in info]))
    print(json.dumps(out))


def _single_summary(name, args):
    """One single-problem workload at its full per-chain length: flips/s,
    effective MH steps/s and the HBM roofline of its step kernel (kernel time
    from HIP events on the context's stream)."""
    wl = _workload(name)
    r = _time_sampler(wl, wl["steps"], 2, 1, "persistent", seed=1, profile=True)
    sec, flips, recs, summ, _, tile, prof = r
    k = _class_rows(prof, 1.0)[0]
    out = {"config": {"workload": wl["desc"], "N": int(wl["Q"].shape[0]), "chains": int(len(wl["betas"])),
                      "mode": wl["mode"], "subset": int(wl["n"] or wl["Q"].shape[0]),
                      "chain_steps_per_step": wl["steps"], "tile": list(tile)},
           "flips_per_s": flips / sec, "effective_mh_steps_per_s": summ / sec, "records_per_s": recs / sec,
           "roofline": {"bound": "hbm", "achieved": k["GB_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": k["hbm_frac"], "traffic": _measured_traffic(name, wl["steps"]),
                        "bytes_per_flip": int(wl["Q"].shape[0] * wl["qbytes"]), "kernel_avg_ms": k["kernel_avg_ms"],
                        "bytes_per_launch": k["bytes_per_launch"]}}
    return out


def _time_sampler(wl, chain_steps: int, steps: int, warmup: int, launch: str, seed: int, tile=(0, 0),
                  profile: bool = False):
    """Returns (seconds per bench step, flips, records and sum M per bench
    step, wall seconds, tile, per-class kernel timing or None)."""
    import torch
    from paper_2210_10513_amd import binding as bd
    from paper_2210_10513_amd.binding import Sampler
    stream = torch.cuda.current_stream()
    s = Sampler(wl["Q"], wl["betas"], wl["n"], wl["mode"], num_chains=len(wl["betas"]), L0=wl["L0"], seed=seed,
                launch=launch, stream=stream, block=tile[0], groups=tile[1])
    for _ in range(warmup):
        s.run(chain_steps)
    s.sync()
    if profile:
        bd.pns_profile(s.ctx, True)
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
    prof = bd.pns_profile_read(s.ctx) if profile else None
    s.close()
    flips = float((st1["flips"] - st0["flips"]).sum()) / steps
    recs = float((st1["steps"] - st0["steps"]).sum()) / steps
    summ = float((st1["sum_M"] - st0["sum_M"]).sum()) / steps
    return ms / 1000.0 / steps, flips, recs, summ, wall, tile, prof


def _cpu_model() -> str:
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_cores() -> int:
    """Cores this process may use, at most 16 (the CPU share of one GPU on a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_tasks(spec):
    """The oracle sample of a workload: (Q as int64/float64, beta, mode, n,
    L0, chain id) per chain.  Batched: one chain of each of 8 problems spread
    evenly over the sizes (smallest and largest included), with the subset
    size the GPU context ran; single problems: 4 chains."""
    import oracle
    modes = {"rf": oracle.MODE_RF, "basic": oracle.MODE_BASIC, "unbiased_sys": oracle.MODE_UNBIASED_SYS}
    tasks = []
    if spec["workload"] == "batched64_uneven_int16":
        from paper_2210_10513_amd import inputs
        Ns = inputs.c4_batched(only=()).extra["Ns"]
        order = np.argsort(Ns, kind="stable")
        pick = [int(order[j]) for j in np.linspace(0, len(order) - 1, 8).round().astype(int)]
        w = inputs.c4_batched(only=pick)
        cp = int(w.extra["chains_per"])
        for i in pick:
            cid = i * cp
            tasks.append((w.Q[i].astype(np.int64), float(w.betas[cid]), modes[w.mode], int(spec["subsets"][i]), w.L0,
                          cid))
    else:
        wl = _workload(spec["workload"])
        Q = wl["Q"].astype(np.int64) if np.issubdtype(wl["Q"].dtype, np.integer) else wl["Q"].astype(np.float64)
        for c in range(4):
            tasks.append((Q, float(wl["betas"][c]), modes[wl["mode"]], int(wl["n"]), wl["L0"], c))
    return tasks


def _cpu_run(tasks, K, offset=0):
    import oracle
    flips = 0
    for Q, beta, mode, n, L0, cid in tasks:
        r = oracle.run(Q, beta, mode, K, n=n, L0=L0, seed=1, num_chains=1,
                       chain_ids=np.array([cid + offset], np.uint32), log=False)
        flips += int(r.flips.sum())
    return flips


_CPU_TASKS = None  # the sample, inherited by the forked workers (not pickled)


def _cpu_worker(args):
    K, offset = args
    return _cpu_run(_CPU_TASKS, K, offset)


def _cpu_baseline_child(spec) -> dict:
    """The single-threaded FP64/int64 oracle on a bounded sample of the
    workload: one core, then one process per core with the chains split
    between them (each process runs the same sample with its own chain ids).
    Runs in a process that never touches the GPU."""
    import multiprocessing as mp
    global _CPU_TASKS
    tasks = _cpu_tasks(spec)
    _CPU_TASKS = tasks
    budget = float(spec.get("budget_s", 12.0))
    # a run costs a fixed part (fields of the initial state, O(N^2)) plus a
    # part per step: time two lengths and size the sample to the budget
    _cpu_run(tasks, 10)  # first call: library load and page faults
    t0 = time.perf_counter()
    _cpu_run(tasks, 20)
    t1 = time.perf_counter()
    _cpu_run(tasks, 60)
    t2 = time.perf_counter()
    per_step = max((t2 - t1) - (t1 - t0), 1e-9) / 40
    fixed = max(0.0, (t1 - t0) - 20 * per_step)
    K = max(20, int((budget - fixed) / per_step))
    t0 = time.perf_counter()
    flips = _cpu_run(tasks, K)
    dt = time.perf_counter() - t0
    cores = _cpu_cores()
    Ns = sorted({int(t[0].shape[0]) for t in tasks})
    sample = (f"{len(tasks)} chains (N = {', '.join(map(str, Ns))}) x {K} steps of the workload, single-threaded "
              f"FP64/int64 oracle ({dt:.1f} s)")
    out = {"value": flips / dt, "unit": "flips/s", "cores": 1, "kind": "oracle", "sample": sample,
           "cpu_model": _cpu_model()}
    if cores > 1:
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(cores) as pool:
            res = pool.map(_cpu_worker, [(K, 1_000_000 * (w + 1)) for w in range(cores)], chunksize=1)
        wall = time.perf_counter() - t0
        out["all_cores"] = {"value": float(sum(res)) / wall, "unit": "flips/s", "cores": cores, "kind": "oracle",
                            "sample": f"{cores} processes, each the sample above with its own chain ids "
                                      f"({wall:.1f} s wall)"}
    return out


def _cpu_baseline(spec) -> dict:
    """Run _cpu_baseline_child in a child process (this process holds the GPU)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline", json.dumps(spec)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-2000:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--cpu-baseline":
        # child process of _cpu_baseline: CPU only, never touches the GPU
        print(json.dumps(_cpu_baseline_child(json.loads(sys.argv[2]))))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched64_uneven_int16")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES; default 12, 8 with --launch graph)")
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
              "(more GPUs would each take their own chains and a copy of Q); use --gpus 1", file=sys.stderr)
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
        _bench_batch(args, wl, cpu_spec=None if args.no_cpu else {"workload": args.workload})
        return
    chain_steps = args.chain_steps or wl["steps"]
    C = len(wl["betas"])
    N = wl["Q"].shape[0]
    tile_req = tuple(int(v) for v in args.tile.split(",")) if args.tile else (0, 0)
    sec, flips, recs, summ, wall, tile, prof = _time_sampler(wl, chain_steps, args.steps, args.warmup, args.launch,
                                                             seed=1, tile=tile_req, profile=True)
    k = _class_rows(prof, 1.0)[0]
    value = flips / sec
    bytes_per_flip = N * wl["qbytes"]
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
        "roofline": {"bound": "hbm", "achieved": k["GB_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": k["hbm_frac"],
                     "traffic": _measured_traffic(args.workload, chain_steps) if args.steps >= 1 else None,
                     "bytes_per_flip": bytes_per_flip, "kernel": "step_kernel",
                     "kernel_avg_ms": k["kernel_avg_ms"], "bytes_per_launch": k["bytes_per_launch"],
                     "timing": "HIP events on the context's stream, every timed step"},
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
        s2, f2, r2, m2, _, t2, _ = _time_sampler(wb, chain_steps // 4, 1, 1, "persistent", seed=2)
        extras["basic64_flips_per_s"] = f2 / s2
        extras["basic64_effective_mh_steps_per_s"] = m2 / s2
        sp, fp, rp, mp, _, _, _ = _time_sampler(wl, 200, 1, 1, "plain", seed=3)
        extras["plain_launch_flips_per_s"] = fp / sp
        extras["persistent_over_plain"] = value / (fp / sp)
        out["variants"] = extras
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline({"workload": args.workload})
    print(json.dumps(out))


if __name__ == "__main__":
    main()
