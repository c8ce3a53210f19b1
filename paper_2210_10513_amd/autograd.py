"""Differentiable log-partition function of a QUBO / Boltzmann model.

For pi_Q(x) = exp(-beta x^T Q x) / Z(Q) over x in {0,1}^N (the Sec 4 target)

    d log Z / d Q_ij = -beta E_pi[x_i x_j]

for every entry of Q, so the gradient is -beta times the second-moment matrix
of the target.  ``LogZ`` estimates it from a jump chain: the forward pass runs
the library's sampler on Q (Rejection-Free by default, or Unbiased PNS) and
keeps snapshots (J_k, M_k) of its records; the backward pass calls the
library's moment kernel, G = X^T diag(m) X on the bf16 matrix cores, and
returns -beta G / sum(m) (the multiplicity-weighted average of Sec 1.2).
With ``weights="rb"`` the multiplicities are replaced by their expected
values given the records (1 / p, or the budget-cut mean for Unbiased PNS):
the ratio estimator of Thm 3 (5) without the sampling noise of M.

The forward value is log Z itself when N <= ``exact_max`` (enumeration on the
device, ``pns_log_partition``).  Beyond that no exact value is available: the
forward returns 0 (so that a loss built on it stays finite and its gradient
flows) -- only the gradient, which is what maximum-likelihood fitting needs,
is meaningful then.

``fit_qubo`` fits Q to data second moments by maximum likelihood: the average
negative log-likelihood of data under pi_Q is beta <Q, E_data[x x^T]> + log Z,
with gradient beta (E_data[x x^T] - E_pi[x x^T]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import binding


@dataclass
class ChainOptions:
    """How LogZ samples: ``num_chains`` chains, ``burn_in`` steps, then
    ``samples`` snapshots every ``every`` steps per chain.  ``weights`` is
    "M" (the sampled multiplicities) or "rb" (their expected values given
    the records, the Rao-Blackwell weights of Thm 3 (5)).  ``state``, if a
    dict, keeps the sampler between calls (warm start, see LogZ)."""
    num_chains: int = 8192
    burn_in: int = 256
    samples: int = 16
    every: int = 8
    mode: str = "rf"
    subset_size: int = 0
    L0: int = 100
    seed: int = 0
    exact_max: int = 24
    weights: str = "M"
    state: Optional[dict] = None


def _sampler_key(N: int, opts: ChainOptions):
    return (N, opts.mode, opts.subset_size, opts.num_chains, opts.L0, opts.every, opts.samples)


class LogZ(torch.autograd.Function):
    """log Z(Q) with the sampled gradient -beta E_pi[x x^T] (see module doc).

    With ``opts.state`` a dict, the sampler context lives in it across calls:
    the next forward only swaps in the new Q (``pns_set_q``: chains keep
    their states, fields and energies are recomputed on the device), clears
    the snapshots and runs ``burn_in + samples * every`` more steps -- a warm
    start with no host-side preparation.  ``release(state)`` frees it."""

    @staticmethod
    def forward(ctx, Q: torch.Tensor, beta: float, opts: ChainOptions):
        if not Q.is_cuda:
            raise ValueError("LogZ needs Q on the GPU")
        N = int(Q.shape[0])
        Qd = Q.detach()
        Qs = ((Qd + Qd.T) * 0.5).to(torch.float32).contiguous()
        stream = torch.cuda.current_stream()
        st = opts.state
        key = _sampler_key(N, opts)
        s = st.get("sampler") if st is not None else None
        if s is not None and st.get("key") == key and st.get("beta") == float(beta):
            s.set_q(Qs)
            s.snapshots_clear()
        else:
            if s is not None:
                s.close()
            s = binding.Sampler(Qs, beta, opts.subset_size, opts.mode, num_chains=opts.num_chains, L0=opts.L0,
                                seed=opts.seed, init="random", launch="persistent", stream=stream,
                                snapshot_every=opts.every, snapshot_capacity=opts.samples)
            if st is not None:
                st.update(sampler=s, key=key, beta=float(beta))
        s.run(opts.burn_in + opts.samples * opts.every)
        value = 0.0  # unknown beyond exact_max: see the module doc
        if N <= opts.exact_max:
            value = binding.pns_log_partition(Qs, beta, stream=stream)
        ctx.sampler = s
        ctx.owned = st is None
        ctx.beta = float(beta)
        ctx.N = N
        ctx.qdtype = Q.dtype
        ctx.rb = _rb(opts)
        return torch.tensor(value, dtype=Q.dtype, device=Q.device)

    @staticmethod
    def backward(ctx, grad_out):
        s = ctx.sampler
        dev = grad_out.device
        G = torch.empty((ctx.N, ctx.N), dtype=torch.float64, device=dev)
        sm = torch.empty(1, dtype=torch.float64, device=dev)
        # -beta * G / sum_w on the device, queued on the sampler's stream
        # (the current stream): no host wait
        binding.pns_logz_grad(s.ctx, 0, ctx.beta, G, sm, rb=ctx.rb)
        grad = G.to(ctx.qdtype)
        if ctx.owned:
            s.close()
        ctx.sampler = None
        return grad_out * grad, None, None


def _rb(opts: ChainOptions) -> bool:
    if opts.weights not in ("M", "rb"):
        raise ValueError("weights must be 'M' or 'rb'")
    return opts.weights == "rb"


def release(state: Optional[dict]) -> None:
    """Free the sampler a LogZ state dict keeps."""
    if state and state.get("sampler") is not None:
        state["sampler"].close()
        state["sampler"] = None
        state["key"] = None


def log_z(Q: torch.Tensor, beta: float, opts: Optional[ChainOptions] = None) -> torch.Tensor:
    return LogZ.apply(Q, beta, opts or ChainOptions())


def moments_of_samples(Q_true: torch.Tensor, beta: float, opts: ChainOptions):
    """(E[x x^T] estimate [N, N] float64 on the device, number of weighted
    records) of pi_{Q_true} from the sampler's snapshots."""
    N = int(Q_true.shape[0])
    Qs = Q_true.detach().to(torch.float32).contiguous()
    s = binding.Sampler(Qs, beta, opts.subset_size, opts.mode, num_chains=opts.num_chains, L0=opts.L0,
                        seed=opts.seed, init="random", launch="persistent", stream=torch.cuda.current_stream(),
                        snapshot_every=opts.every, snapshot_capacity=opts.samples)
    s.run(opts.burn_in + opts.samples * opts.every)
    G = torch.empty((N, N), dtype=torch.float64, device=Q_true.device)
    sm = torch.empty(1, dtype=torch.float64, device=Q_true.device)
    binding.pns_snapshot_moments(s.ctx, 0, G, sum_m=sm, rb=_rb(opts))
    out = G / sm
    s.close()
    return out, opts.num_chains * opts.samples


@dataclass
class FitResult:
    Q: torch.Tensor
    moment_gap: list = field(default_factory=list)   # max |E_data - E_model| per iteration (sampled)
    loss: list = field(default_factory=list)         # NLL when log Z is exact, else NaN


def fit_qubo(data_moments: torch.Tensor, beta: float, iters: int, lr: float, opts: ChainOptions,
             Q0: Optional[torch.Tensor] = None, momentum: float = 0.9, centered: bool = True,
             average_from: Optional[int] = None) -> FitResult:
    """Maximum-likelihood fit of Q to data second moments D = E_data[x x^T]
    by gradient descent with momentum on beta <Q, D> + log Z(Q); every
    gradient of log Z comes from LogZ's backward (sampled moments on the
    matrix cores).

    With ``centered`` (default) the descent runs in centered coordinates:
    Q_ij = W_ij off the diagonal and Q_ii = a_i - 2 sum_{j != i} W_ij mu_j
    with mu = diag(D) (the data means), i.e. the energy is written as
    (x - mu)^T W (x - mu) + a^T x + const.  The optimum is the
    same (a fixed linear change of coordinates), but the gradient in W is
    the difference of covariances instead of second moments, which removes
    the collective direction driven by the means whose curvature grows like
    N and would force a step size ~ 1/N.

    With ``average_from`` = t0 the result is the mean of the iterates after
    the updates t0 .. iters-1 (tail averaging of Polyak and Juditsky, 1992)
    instead of the last iterate: every gradient is a Monte Carlo estimate,
    and the last iterate keeps the noise of its last steps, which the mean
    averages out."""
    D = data_moments.to(torch.float32)
    N = int(D.shape[0])
    dev = D.device
    eye = torch.eye(N, device=dev)
    mu = torch.diagonal(D).clone()
    Qinit = (torch.zeros((N, N), dtype=torch.float32, device=dev) if Q0 is None else Q0.clone().float())
    if centered:
        W = (Qinit * (1 - eye)).clone().requires_grad_(True)
        a = (torch.diagonal(Qinit) + 2 * (Qinit * (1 - eye)) @ mu).clone().requires_grad_(True)
        params = [W, a]
    else:
        Qp = Qinit.clone().requires_grad_(True)
        params = [Qp]

    def build_q():
        if centered:
            Ws = (W + W.T) * 0.5 * (1 - eye)
            return Ws + torch.diag(a - 2 * (Ws @ mu))
        return (Qp + Qp.T) * 0.5

    if average_from is not None and not 0 <= average_from < iters:
        raise ValueError(f"average_from must lie in [0, {iters})")
    vel = [torch.zeros_like(p) for p in params]
    res = FitResult(Q=Qinit)
    Qsum, nsum = None, 0
    state = opts.state if opts.state is not None else {}
    o = ChainOptions(**{**opts.__dict__, "state": state})
    try:
        for it in range(iters):
            Q = build_q()
            lz = LogZ.apply(Q, beta, o)
            loss = beta * (Q * D).sum() + lz
            for p in params:
                p.grad = None
            Q.retain_grad()
            loss.backward()
            with torch.no_grad():
                res.moment_gap.append(float(Q.grad.abs().max().item() / beta))
                res.loss.append(float(loss.item()) if N <= o.exact_max else float("nan"))
                for p, v in zip(params, vel):
                    v.mul_(momentum).add_(p.grad)
                    p.sub_(lr * v)
                if average_from is not None and it >= average_from:
                    Qi = build_q()
                    Qsum = Qi.clone() if Qsum is None else Qsum.add_(Qi)
                    nsum += 1
    finally:
        if opts.state is None:
            release(state)
    with torch.no_grad():
        res.Q = build_q().detach() if Qsum is None else Qsum / nsum
    return res
