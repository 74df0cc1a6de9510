"""SMC driver over the C ABI (Sec. "Algorithm and implementation").

A prior-start run draws N particles from the prior (K uniform on [k_lo, k_hi], each
component uniform in the prior box) at beta = 0 and repeats until beta = 1:

1. choose the next beta by the ESS condition (eq. ess_target) and reweight
   (eq. incremental_weight), accumulating the evidence: ``smcx_next_beta``;
2. resample systematically by the normalised weights: ``smcx_resample_systematic``;
3. mutate every particle ``n_mutations`` times with the mixture kernel of
   eq. kernel_mixture: with probability p_nuts a NUTS transition of the
   tempered target (``smcx_nuts_transition`` with a mask), otherwise a birth
   (a component drawn from the prior) or the death of a uniformly chosen
   component, scored by ``delta_logl_birth_death`` and accepted or rejected
   by ``smcx_rj_apply``.

With ``metric=True`` the NUTS moves use a mass matrix from the Hessian of
the negative log posterior (Sec. "No-U-Turn-Sampler"), fixed for the whole
population during each mutation step so that the move leaves the tempered
target invariant: before the step the Gauss-Newton blocks of every
component are computed at the population's positions
(``smcx_gauss_newton_metric_blocks``), averaged into one P x P block
(``smcx_metric_pool_blocks``), floored by the prior's precision
12 / width^2 on the diagonal and factored (``smcx_metric_factor_blocks``);
every component of every particle then moves with that block in the
whitened momentum (``smcx_nuts_transition_metric_blocks``) with the step
``eps_metric``. A matrix taken at each particle's own position would adapt
to it better but would not leave the target invariant (the reverse move
would use the matrix at the end point).

The posterior-start mode (``run_posterior_start``) starts instead from a
population sampled on the first `split` samples of the data and follows the
bridge of eq. reuse_bridge: the problem's bridge split makes every tempered
call evaluate logL[0, split) + beta logL[split, T), and the incremental
weights use the untempered log-likelihood of the new samples only. For the
frequency-domain Galactic binaries, whose bins all change when the record
grows, ``run_bridge_start`` bridges two handles instead:
(1 - beta) logL_short + beta logL_long.

All arithmetic runs in the library's kernels. This module draws the random
inputs on the device (a seeded torch generator) and sequences the calls; it
synchronises with the host a few times per iteration (to read beta and the
new row count).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import torch

from . import smcx


@dataclass
class SMCConfig:
    N: int
    k_lo: int = 1
    k_hi: int = 10
    alpha: float = 0.9                 # ESS fraction kept per iteration
    p_nuts: float = 0.6                # mixture weights of eq. kernel_mixture
    p_birth: float = 0.2
    p_death: float = 0.2
    n_mutations: int = 4               # mixture-kernel steps per SMC iteration
    max_depth: int = 6                 # NUTS tree depth
    # NUTS step size as a function of beta (identity metric in raw coordinates);
    # the default suits the prior bridge, whose target widens as beta falls
    eps: Callable[[float], float] = field(default=lambda beta: 3e-4 / math.sqrt(max(beta, 1e-4)))
    max_iters: int = 200
    seed: int = 0
    metric: bool = False               # NUTS with the Gauss-Newton mass matrix
    eps_metric: float = 0.3            # its step size (whitened units)
    ridge: Optional[Sequence[float]] = None  # diagonal floor per parameter; None: 12 / width^2


@dataclass
class SMCResult:
    offsets: torch.Tensor              # final population (CSR), on the device
    theta: torch.Tensor
    betas: list
    ess: list
    log_evidence: float                # sum of the log Z increments
    k_hist: list                       # per iteration: counts of K = 0..k_hi after mutation
    rj_accept: list                    # per iteration: accepted fraction of birth/death moves
    nuts_steps: list                   # per iteration: leapfrog steps of the NUTS moves

    @property
    def iterations(self) -> int:
        return len(self.betas)


def run_prior_start(prob: smcx.Problem, prior_lo: torch.Tensor, prior_hi: torch.Tensor,
                    cfg: SMCConfig, on_iteration: Optional[Callable[[int, dict], None]] = None
                    ) -> SMCResult:
    """Run the prior-start SMC of the paper's Sec. "Algorithm and implementation"
    on the problem's data. The handle needs n_max >= N, k_max >= k_hi and
    m_max >= N k_hi; prior_lo, prior_hi are the [P] box of the uniform prior
    (on the device)."""
    _check(prob, cfg)
    gen = _generator(prior_lo.device, cfg.seed)
    N = cfg.N
    K = torch.randint(cfg.k_lo, cfg.k_hi + 1, (N,), generator=gen, device=prior_lo.device)
    off = torch.zeros(N + 1, dtype=torch.int64, device=prior_lo.device)
    off[1:] = torch.cumsum(K, 0)
    th = _prior_rows(prob, prior_lo, prior_hi, int(off[-1]), gen)
    prob.set_bridge_split(0)
    return _run(prob, off, th, prior_lo, prior_hi, cfg, gen,
                lambda o, t: smcx.logl_batch(prob, o, t), on_iteration)


def run_posterior_start(prob: smcx.Problem, split: int, offsets: torch.Tensor,
                        theta: torch.Tensor, prior_lo: torch.Tensor, prior_hi: torch.Tensor,
                        cfg: SMCConfig, on_iteration: Optional[Callable[[int, dict], None]] = None
                        ) -> SMCResult:
    """Run the posterior-start SMC (eq. reuse_bridge): `offsets`, `theta` are
    a population sampled from the posterior on the first `split` samples of
    the problem's data (on the same time grid), for example the result of
    run_prior_start on a problem built from them. The bridge split is set on
    the handle for the run and cleared afterwards."""
    _check(prob, cfg)
    if not 0 < split < prob.T:
        raise ValueError("split must lie inside the data")
    if offsets.numel() - 1 != cfg.N:
        raise ValueError("the starting population must have cfg.N particles")
    gen = _generator(prior_lo.device, cfg.seed)
    prob.set_bridge_split(split)
    try:
        return _run(prob, offsets, theta.contiguous(), prior_lo, prior_hi, cfg, gen,
                    lambda o, t: smcx.reweight_extend(prob, split, prob.T, o, t, 0.0)[0],
                    on_iteration)
    finally:
        prob.set_bridge_split(0)


def run_bridge_start(prob: smcx.Problem, partner: smcx.Problem, offsets: torch.Tensor,
                     theta: torch.Tensor, prior_lo: torch.Tensor, prior_hi: torch.Tensor,
                     cfg: SMCConfig, on_iteration: Optional[Callable[[int, dict], None]] = None
                     ) -> SMCResult:
    """Posterior-start across two frequency-domain records (eq. reuse_bridge):
    `offsets`, `theta` sample the posterior on the shorter record held by
    `partner`; the run follows (1 - beta) logL_partner + beta logL_prob from
    beta = 0 to 1, with incremental weights from logL_prob - logL_partner. The
    handles' bridge is set for the run and cleared afterwards."""
    _check(prob, cfg)
    if offsets.numel() - 1 != cfg.N:
        raise ValueError("the starting population must have cfg.N particles")
    gen = _generator(prior_lo.device, cfg.seed)
    prob.set_bridge_partner(partner)
    try:
        return _run(prob, offsets, theta.contiguous(), prior_lo, prior_hi, cfg, gen,
                    lambda o, t: smcx.logl_batch(prob, o, t) - smcx.logl_batch(partner, o, t),
                    on_iteration)
    finally:
        prob.set_bridge_partner(None)


def _check(prob: smcx.Problem, cfg: SMCConfig) -> None:
    if not (cfg.N <= prob.n_max and cfg.k_hi <= prob.k_max and cfg.N * cfg.k_hi <= prob.m_max):
        raise ValueError("the problem handle is too small for this SMC configuration")
    if abs(cfg.p_nuts + cfg.p_birth + cfg.p_death - 1.0) > 1e-12:
        raise ValueError("mixture weights must sum to 1")
    if cfg.metric and cfg.k_hi * prob.P > 128:
        raise ValueError("the NUTS metric needs k_hi * P <= 128")


def _generator(dev, seed: int) -> torch.Generator:
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    return gen


def _prior_rows(prob, lo, hi, n: int, gen) -> torch.Tensor:
    lo, hi = lo.to(torch.float64), hi.to(torch.float64)
    u = torch.rand((n, prob.P), generator=gen, dtype=torch.float64, device=lo.device)
    return (lo + u * (hi - lo)).contiguous()


def _run(prob, off, th, prior_lo, prior_hi, cfg, gen, weight_logl, on_iteration) -> SMCResult:
    """The SMC iterations from beta = 0; weight_logl(offsets, theta) gives the
    untempered log-likelihood whose (beta - beta_prev) multiple is the log
    incremental weight."""
    dev = prior_lo.device
    P, N, D = prob.P, cfg.N, cfg.max_depth
    smcx.nuts_reserve(prob, D)
    lo, hi = prior_lo.to(torch.float64).contiguous(), prior_hi.to(torch.float64).contiguous()
    f64 = dict(dtype=torch.float64, device=dev)
    M = int(off[-1])
    log_ratio = math.log(cfg.p_death / cfg.p_birth)
    if cfg.metric:
        ridge = (list(cfg.ridge) if cfg.ridge is not None
                 else (12.0 / (hi - lo) ** 2).cpu().tolist())
        fbuf = torch.empty((N * cfg.k_hi, P, P), **f64)
        wbuf = torch.empty_like(fbuf)
        fmean = torch.empty((1, P, P), **f64)
    beta = 0.0
    res = SMCResult(off, th, [], [], 0.0, [], [], [])
    for it in range(cfg.max_iters):
        logl = weight_logl(off, th)
        beta_arr, _, w_norm, sc = smcx.next_beta(prob, logl, beta, cfg.alpha)
        beta, ess, dlogz = (float(x) for x in sc[:3].cpu())
        res.betas.append(beta)
        res.ess.append(ess)
        res.log_evidence += dlogz
        u = float(torch.rand(1, generator=gen, **f64))
        _, off, th_all = smcx.resample_systematic(prob, off, th, w_norm, u, m_cap=N * cfg.k_hi)
        M = int(off[-1])
        th = th_all[:M]
        acc_rj = tried_rj = steps = 0
        eps = cfg.eps_metric if cfg.metric else float(cfg.eps(beta))
        for _ in range(cfg.n_mutations):
            r = torch.rand(N, generator=gen, **f64)
            nuts = r < cfg.p_nuts
            move = torch.where(nuts, 0, torch.where(r < cfg.p_nuts + cfg.p_birth, 1, 2)).to(torch.int8)
            if M > 0:
                nuts_u8 = nuts.to(torch.uint8)
                # the NUTS move starts from the gradient of the particles it moves
                l, g = smcx.logl_grad_batch(prob, off, th, beta_arr, mask=nuts_u8)
                mom = torch.randn((M, P), generator=gen, **f64)
                dirs = (torch.randint(0, 2, (N, D), generator=gen, device=dev) * 2 - 1).to(torch.int8)
                ul = torch.rand((N, (1 << D) - 1), generator=gen, **f64)
                ut = torch.rand((N, D), generator=gen, **f64)
                wblocks = None
                if cfg.metric:
                    # one block for the whole population, fixed for this step
                    F = smcx.gauss_newton_metric_blocks(prob, off, th, beta_arr, out=fbuf[:M])
                    smcx.metric_pool_blocks(prob, F, M=M, out=fmean[0])
                    smcx.metric_factor_blocks(prob, fmean, ridge, out=fmean, M=1)
                    wblocks = wbuf[:M]
                    wblocks.copy_(fmean.expand(M, P, P))
                _, st, _ = smcx.nuts_transition(prob, off, beta_arr, eps, D, th, l, g, mom, dirs,
                                                ul, ut, lo, hi, mask=nuts_u8,
                                                metric_blocks=wblocks)
                steps += int(st.sum())
            Kc = off[1:] - off[:-1]
            tb = _prior_rows(prob, lo, hi, N, gen)
            di = torch.floor(torch.rand(N, generator=gen, **f64) * Kc).to(torch.int32)
            # the death overlap only where a death is proposed (-1: none)
            di = torch.where((Kc > 0) & (move == 2), di, torch.full_like(di, -1))
            # scored only for the particles that propose a birth or a death
            db, dd = smcx.delta_logl_birth_death(prob, off, th, beta_arr, tb, di,
                                                 mask=(move != 0).to(torch.uint8))
            log_u = torch.log(torch.rand(N, generator=gen, **f64))
            acc, off, th_all = smcx.rj_apply(prob, off, th, move, tb, di, db, dd, log_u, cfg.k_lo,
                                             cfg.k_hi, log_ratio, m_cap=M + N)
            M = int(off[-1])
            th = th_all[:M]
            acc_rj += int(acc.sum())
            tried_rj += int((~nuts).sum())
        Kc = (off[1:] - off[:-1]).cpu()
        res.k_hist.append(torch.bincount(Kc, minlength=cfg.k_hi + 1).tolist())
        res.rj_accept.append(acc_rj / max(tried_rj, 1))
        res.nuts_steps.append(steps)
        if on_iteration:
            on_iteration(it, dict(beta=beta, ess=ess, k_hist=res.k_hist[-1],
                                  rj_accept=res.rj_accept[-1], nuts_steps=steps))
        if beta >= 1.0:
            break
    prob.device_status()
    res.offsets, res.theta = off, th
    return res
