"""Differentiable log-partition function of a QUBO / Boltzmann model.

For pi_Q(x) = exp(-beta x^T Q x) / Z(Q) over x in {0,1}^N (the Sec 4 target)

    d log Z / d Q_ij = -beta E_pi[x_i x_j]

for every entry of Q, so the gradient is -beta times the second-moment matrix
of the target.  ``LogZ`` estimates it from a jump chain: the forward pass runs
the library's sampler on Q (Rejection-Free by default, or Unbiased PNS) and
keeps snapshots (J_k, M_k) of its records; the backward pass calls the
library's moment kernel, G = X^T diag(m) X on the bf16 matrix cores, and
returns -beta G / sum(m) (the multiplicity-weighted average of Sec 1.2).

The forward value is log Z itself when N <= ``exact_max`` (enumeration on the
device, ``pns_log_partition``); beyond that no exact value is available and
the forward returns NaN -- the gradient, which is what maximum-likelihood
fitting needs, is still the sampled estimate.

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
    ``samples`` snapshots every ``every`` steps per chain.  ``state``, if a
    dict, carries the chains' final states between calls (warm start)."""
    num_chains: int = 8192
    burn_in: int = 256
    samples: int = 16
    every: int = 8
    mode: str = "rf"
    subset_size: int = 0
    L0: int = 100
    seed: int = 0
    exact_max: int = 24
    state: Optional[dict] = None


class LogZ(torch.autograd.Function):
    """log Z(Q) with the sampled gradient -beta E_pi[x x^T] (see module doc)."""

    @staticmethod
    def forward(ctx, Q: torch.Tensor, beta: float, opts: ChainOptions):
        if not Q.is_cuda:
            raise ValueError("LogZ needs Q on the GPU")
        N = int(Q.shape[0])
        Qd = Q.detach()
        Qs = ((Qd + Qd.T) * 0.5).to(torch.float32).contiguous()
        stream = torch.cuda.current_stream()
        x0 = None
        init = "random"
        if opts.state is not None and "x" in opts.state:
            x0 = opts.state["x"]
        s = binding.Sampler(Qs, beta, opts.subset_size, opts.mode, num_chains=opts.num_chains, L0=opts.L0,
                            seed=opts.seed, init=init, x0=x0, launch="persistent", stream=stream,
                            snapshot_every=opts.every, snapshot_capacity=opts.samples)
        s.run(opts.burn_in + opts.samples * opts.every)
        if opts.state is not None:
            opts.state["x"] = s.read_current()["x"]
            opts.state["seed_step"] = opts.state.get("seed_step", 0) + 1
        value = float("nan")
        if N <= opts.exact_max:
            value = binding.pns_log_partition(Qs, beta, stream=stream)
        ctx.sampler = s
        ctx.beta = float(beta)
        ctx.N = N
        ctx.qdtype = Q.dtype
        return torch.tensor(value, dtype=Q.dtype, device=Q.device)

    @staticmethod
    def backward(ctx, grad_out):
        s = ctx.sampler
        dev = grad_out.device
        G = torch.empty((ctx.N, ctx.N), dtype=torch.float64, device=dev)
        sm = binding.pns_snapshot_moments(s.ctx, 0, G)
        s.close()
        ctx.sampler = None
        if sm <= 0:
            raise RuntimeError("no snapshot carries weight: run more steps")
        grad = (G * (-ctx.beta / sm)).to(ctx.qdtype)
        return grad_out * grad, None, None


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
    sm = binding.pns_snapshot_moments(s.ctx, 0, G)
    s.close()
    return G / sm, opts.num_chains * opts.samples


@dataclass
class FitResult:
    Q: torch.Tensor
    moment_gap: list = field(default_factory=list)   # max |E_data - E_model| per iteration (sampled)
    loss: list = field(default_factory=list)         # NLL when log Z is exact, else NaN


def fit_qubo(data_moments: torch.Tensor, beta: float, iters: int, lr: float, opts: ChainOptions,
             Q0: Optional[torch.Tensor] = None, momentum: float = 0.9) -> FitResult:
    """Maximum-likelihood fit of Q to data second moments by gradient descent
    with momentum on beta <Q, D> + log Z(Q); every gradient of log Z comes
    from LogZ's backward (sampled moments on the matrix cores)."""
    D = data_moments.to(torch.float32)
    N = int(D.shape[0])
    Q = (torch.zeros((N, N), dtype=torch.float32, device=D.device) if Q0 is None else Q0.clone().float())
    Q.requires_grad_(True)
    vel = torch.zeros_like(Q)
    res = FitResult(Q=Q)
    state = opts.state if opts.state is not None else {}
    for it in range(iters):
        o = ChainOptions(**{**opts.__dict__, "seed": opts.seed + 7919 * (it + 1), "state": state})
        lz = LogZ.apply(Q, beta, o)
        loss = beta * (Q * D).sum() + lz
        if Q.grad is not None:
            Q.grad = None
        loss.backward()
        with torch.no_grad():
            g = Q.grad
            res.moment_gap.append(float((g.abs().max() / beta).item()))
            res.loss.append(float(loss.item()) if not math.isnan(float(lz.item())) else float("nan"))
            vel.mul_(momentum).add_(g)
            Q.sub_(lr * vel)
            Q.copy_((Q + Q.T) * 0.5)
    res.Q = Q.detach()
    return res
