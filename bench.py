#!/usr/bin/env python3
"""Throughput of the batched population likelihood paths on one MI355X.

Default workload (gb_grad, the largest logL + gradient configuration: chirping
sinusoids, T = 2^17 samples, N = 4096 particles, K ~ U{0..30}): a step is one
logl_grad_batch call over the whole population (template synthesis with the
phase in FP64, residual, FP64 inner products, adjoint gradient and ragged
batching in one fused pass); the unit of work is one particle log-likelihood
+ gradient evaluation. The same population is then run through the plain
one-particle-per-launch FP64 form on the same GPU, and through the FP64 CPU
oracle on a bounded sample on the host cores (all threads, then one thread);
the oracle's results on that sample also give the reported error of both GPU
forms. The Gaussian-pulse population (pulse_batch: T = 4096, N = 16384,
K ~ U{0..20}, beta ~ U[0,1]) is measured the same way and attached as
"secondary", its accuracy over every particle. Inputs are seeded synthetic
workloads resident in device memory before the timed region starts.

Other workloads (--workload):
  pulse_batch   the pulse population alone
  gb_extend     data-assimilation reweighting: segment logL of every particle
                on the new samples plus weights, ESS and evidence increment
  pulse_mutate  one NUTS transition of every particle (hipGraph-replayed
                leapfrog sweeps) plus the birth/death log-likelihood changes
  smc_pulses    whole SMC runs with NUTS on the Gauss-Newton mass matrix
                (prior-start, timed per run; then one posterior-start run, and
                one identity-metric run for comparison) on a 10-pulse problem
                at N = 6000
  metric        Gauss-Newton metric of the pulse population (matrix cores)
  gb_lisa       LISA Galactic binaries in the frequency domain (A+E, FP64),
                N = 40000, one logL+grad call per step
  smc_gblisa    whole prior-start SMC runs on ten Galactic binaries, N = 40000

Prints one JSON line. Usage: python bench.py [--steps K] [--warmup W]
[--workload ...] [--gpus 1].
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle logL+grad evals/sec (ragged K) vs plain GPU form at ≤1e-6 rel err"

# MI355X: 256 CUs at 2.4 GHz, four SIMDs per CU. The published FP32 vector
# peak, 157.3 TFLOP/s, counts packed FP32 FMAs (two per lane and cycle);
# the library is compiled with packed FP32 instructions disabled, and the issue
# probe (--workload issue_probe) measures what the vector units then do per
# CU and clock: 63 lanes of v_fmac_f32 / v_fma_f32 (of 64), 96-105 of
# v_mul_f32 / v_add_f32 / v_add_u32 (of 128), 58 of v_cvt_f32_i32 (of 64), 30
# of v_exp_f32 / v_sin_f32 (of 32), 61 of v_alignbit_b32 (of 64) and 50 of
# v_fma_f64 (of 64). So the FP32
# ceiling without packed instructions is 64 FMA lanes per CU and clock:
PEAK_FP32_TFLOPS = 78.6          # 256 CUs x 64 lanes x 2 flops x 2.4 GHz
PUBLISHED_FP32_TFLOPS = 157.3    # with packed FP32 FMAs (which the library does not emit)
CLOCK_HZ = 2.4e9

# Issue cost of one component-sample in FP32-FMA slots (one slot = one lane
# of a full-rate FMA issue): FMA, conversion and funnel shift 1, two-operand
# multiply or add (FP32 or integer) 1/2, from the rates above, and a
# transcendental 1, the issue slot it takes from the other vector work. A
# stream of transcendentals alone runs at their own unit's rate (two slots
# each), but in these kernels that unit overlaps with the rest: charged at
# two slots, the forward-only sinusoid pass would run at 1.04 of the
# ceiling, and the counters put the unit's busy share at 15-34% of the
# kernels' time, so it is never the limit. The operations are those the
# method needs per component-sample:
#   pulse forward: add, fmac, mul, exp2, fmac                          4
#   pulse adjoint: add, fmac, mul, exp2, mul, add, fmac, fmac          6
#   sinusoid forward: in groups of four samples, two sines from the
#                     phase (int add, one funnel shift, sin: 2.5 each),
#                     two by the three-term relation (fma: 1 each),
#                     and four fmac                          (5 + 2 + 4) / 4
#   sinusoid adjoint: the phasor in groups of four samples, the first
#                     turned from the previous group's first and the
#                     second from the first by complex multiplies (mul,
#                     fma, mul, fma: 3 each), the other two by the
#                     three-term recurrence (fma, fma: 2 each), the
#                     tile's first from sin and cos (funnel shift, sin,
#                     cos: 3); then fmac, fmac, add, add              5.5
# (sinusoids with the linear tile phase, which the workloads' chirps take;
# the adjoint's three moment sums are running sums)
SLOTS = {(0, "grad"): 10.0, (1, "grad"): 2.75 + 5.5, (0, "fwd"): 4.0, (1, "fwd"): 2.75}


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs, scaled by the same counters' readings for a device copy of
# known size. Valid only for the kernel source they were taken on (its hash).
PMC_TRAFFIC = {("gb_grad", "32,16384,1"): {"bytes": 2.4607e+07, "kernels_sha1": "bca9d37ca926281b"},
               ("pulse_batch", "64,4096,1"): {"bytes": 1.3133e+07, "kernels_sha1": "bca9d37ca926281b"}}


def kernels_sha1():
    import hashlib
    path = os.path.join(ROOT, "paper_2609_17674_amd", "csrc", "smcx_kernels.hip")
    return hashlib.sha1(open(path, "rb").read()).hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def roofline(model, kind, comp_samples, kern_ms, kernel):
    """ALU roofline of the population kernel: its algorithmic work in FP32-FMA
    slots (times 2 flops) per launch over the launch's time, against the FP32
    FMA ceiling without packed instructions; the fraction of the published
    (packed) figure is given beside it."""
    per = SLOTS[(model, kind)]
    slots = per * comp_samples
    achieved = 2.0 * slots / (kern_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": kernel, "kernel_ms": round(kern_ms, 5),
            "work": f"{comp_samples:.4e} component-samples x {per:g} "
                    f"FP32-FMA slots x 2 flops",
            "peak_basis": "FP32 FMA issue without packed instructions (64 lanes/CU/clock, "
                          "measured 63 by the issue probe)",
            "frac_of_published_fp32": round(achieved / PUBLISHED_FP32_TFLOPS, 4)}


def component_samples(w, s_lo, s_hi):
    """Component-samples the method needs on samples [s_lo, s_hi). Sinusoids
    cover every sample; pulses are truncated where |t - t0| >= sqrt(128 ln 2) w
    (template below 2^-64 of its peak), so only samples inside that support
    count."""
    import numpy as np
    if w.model != 0:
        return float(w.M) * (s_hi - s_lo)
    c = (w.theta[:, 1] - w.t_start) / w.dt
    hw = np.sqrt(128.0 * np.log(2.0)) * np.abs(w.theta[:, 2]) / w.dt
    lo = np.maximum(np.ceil(c - hw), s_lo)
    hi = np.minimum(np.floor(c + hw), s_hi - 1)
    return float(np.maximum(hi - lo + 1.0, 0.0).sum())


def timed(fn, prob, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    prob.device_status()
    prob.profile_begin(max(steps, 1) * 300)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, kern_n = prob.profile_end()
    return (t1 - t0) * 1e3 / steps, kern_ms / max(kern_n, 1), kern_n


def cpu_sample(w, per_eval_fn, budget_s, rng):
    import numpy as np
    from paper_2609_17674_amd import workloads as wl
    probe = wl.subsample(w, np.sort(rng.choice(w.N, size=min(32, w.N), replace=False)))
    t0 = time.perf_counter()
    per_eval_fn(probe)
    per = (time.perf_counter() - t0) / probe.N
    n = int(min(w.N, max(64, budget_s / max(per, 1e-9))))
    idx = np.sort(rng.choice(w.N, size=n, replace=False))
    return idx, wl.subsample(w, idx)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def setup(w, dev, smcx, torch):
    inj = torch.tensor(w.inj, device=dev)
    d = torch.tensor(w.noise, device=dev) + smcx.template_sum(w.model, inj, w.T, w.t_start, w.dt)
    prob = smcx.Problem(w.model, d, w.t_start, w.dt, w.sigma, w.k_max, w.N, w.M)
    return d, prob, torch.tensor(w.offsets, device=dev), torch.tensor(w.theta, device=dev)


def bench_grad(args, w, dev, smcx, np, torch, cpu_seconds, cpu1_seconds, check_all=False):
    """One logl_grad_batch call over the population per step. Besides the
    timed value: the plain one-particle-per-launch FP64 form over the whole
    population, the oracle on a bounded sample (all host threads, then one
    thread on a smaller sample), and the error of both GPU forms against the
    oracle on that sample (the whole population with check_all)."""
    d, prob, off, th = setup(w, dev, smcx, torch)
    beta = torch.tensor(w.beta, device=dev)
    logl = torch.empty(w.N, dtype=torch.float64, device=dev)
    grad = torch.empty_like(th)
    if args.tiling:
        S, chunk, so = (int(x) for x in args.tiling.split(","))
        prob.set_tiling(smcx.KIND_GRAD, S, chunk, so)
        tuned = (S, chunk, so, float("nan"))
    else:
        tuned = prob.autotune(smcx.KIND_GRAD, off, th, beta, reps=5)
    log(f"[bench] {w.name}: tiling S={tuned[0]} chunk={tuned[1]} sorted={tuned[2]} "
        f"({tuned[3]:.4f} ms/call when tuned)")

    def step():
        smcx.logl_grad_batch(prob, off, th, beta, logl=logl, grad=grad)

    ms, kern_ms, _ = timed(step, prob, args.steps, args.warmup)
    value = w.N / (ms * 1e-3)
    log(f"[bench] {w.name}: {ms:.4f} ms/step, pop_kernel {kern_ms:.4f} ms, {value:.4e} evals/s")
    rl = roofline(w.model, "grad", component_samples(w, 0, w.T), kern_ms,
                  f"pop_kernel<{w.model},{tuned[0]},true,{'true' if tuned[2] == 2 else 'false'}> "
                  f"(fused forward+adjoint)")
    pmc = PMC_TRAFFIC.get((w.name, f"{tuned[0]},{tuned[1]},{tuned[2]}"))
    if pmc and pmc["kernels_sha1"] == kernels_sha1():
        rl["traffic"] = pmc["bytes"]
    out_l, out_g = logl.cpu().numpy(), grad.cpu().numpy()

    plain = None
    if not args.no_plain:
        pl, pg = torch.empty_like(logl), torch.empty_like(grad)
        sub = min(64, w.N)
        msub = int(w.offsets[sub])
        smcx.plain_logl_grad(prob, w.offsets[:sub + 1], th[:msub], beta[:sub], logl=pl[:sub],
                             grad=pg[:msub])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smcx.plain_logl_grad(prob, w.offsets, th, beta, logl=pl, grad=pg)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3
        plain = {"value": w.N / (plain_ms * 1e-3), "unit": "evals/s", "ms_per_step": plain_ms,
                 "form": "one particle per forward+adjoint launch pair, FP64"}
        plain_l, plain_g = pl.cpu().numpy(), pg.cpu().numpy()
        log(f"[bench] {w.name}: plain form {plain_ms:.1f} ms/step")

    cpu = accuracy = None
    if not args.no_cpu_baseline:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import parity as pm
        oracle.build(force=False)
        d_host = d.cpu().numpy()
        rng = np.random.default_rng(2024)

        def orc(s):
            return oracle.logl_grad(w.model, d_host, w.t_start, w.dt, w.sigma, s.offsets, s.theta,
                                    s.beta)

        if check_all:
            idx = np.arange(w.N)
            sub = w
        else:
            idx, sub = cpu_sample(w, orc, cpu_seconds, rng)
        threads = oracle.get_threads()
        t0 = time.perf_counter()
        ref_l, ref_g = orc(sub)
        cpu_s = time.perf_counter() - t0
        n = len(idx)
        # one host thread on a smaller sample of the same workload
        oracle.set_threads(1)
        try:
            idx1, sub1 = cpu_sample(w, orc, cpu1_seconds, np.random.default_rng(2026))
            t0 = time.perf_counter()
            orc(sub1)
            cpu1_s = time.perf_counter() - t0
        finally:
            oracle.set_threads(threads)
        cpu = {"value": n / cpu_s, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"{n} of {w.N} particles of the same workload (seeded), all {w.T} "
                         f"samples, {cpu_s:.1f} s on {threads} threads",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "value_1_thread": len(idx1) / cpu1_s,
               "sample_1_thread": f"{len(idx1)} particles, {cpu1_s:.1f} s"}
        log(f"[bench] {w.name}: cpu oracle {n} particles in {cpu_s:.1f} s ({threads} threads), "
            f"{len(idx1)} in {cpu1_s:.1f} s (1 thread)")
        rows = np.concatenate([np.arange(w.offsets[i], w.offsets[i + 1]) for i in idx])
        el = pm.logl_errors(out_l[idx], ref_l)
        rel, cos = pm.grad_errors(w.model, sub.offsets, sub.theta, out_g[rows], ref_g, w.T, w.dt)
        Ks = np.diff(w.offsets)[idx]
        accuracy = {"checked_particles": n, "max_K_checked": int(Ks.max()),
                    "logl_max_rel_err": float(el.max()),
                    "logl_p99_rel_err": float(np.percentile(el, 99)),
                    "grad_max_rel_err": float(rel.max()) if len(rel) else 0.0,
                    "grad_p99_rel_err": float(np.percentile(rel, 99)) if len(rel) else 0.0,
                    "grad_min_cos": float(cos.min()) if len(cos) else 1.0}
        if plain is not None:
            pel = pm.logl_errors(plain_l[idx], ref_l)
            prel, _ = pm.grad_errors(w.model, sub.offsets, sub.theta, plain_g[rows], ref_g, w.T,
                                     w.dt)
            plain["logl_max_rel_err"] = float(pel.max())
            plain["grad_max_rel_err"] = float(prel.max()) if len(prel) else 0.0
    return dict(metric=METRIC, value=value, unit="evals/s", ms_per_step=ms,
                config={"workload": w.name, "T": w.T, "N": w.N, "M": w.M,
                        "K": f"U{{0..{w.k_max}}}",
                        "beta": "U[0,1]" if w.name == "pulse_batch" else "1",
                        "tiling": {"S": tuned[0], "chunk_len": tuned[1], "sorted": tuned[2]}},
                plain_gpu=plain, speedup_vs_plain=(value / plain["value"]) if plain else None,
                accuracy=accuracy, roofline=rl, cpu_baseline=cpu)


def bench_extend(args, w, dev, smcx, np, torch):
    T1, T2 = w.extra["T1"], w.extra["T2"]
    d, prob, off, th = setup(w, dev, smcx, torch)
    if args.tiling:
        S, chunk, so = (int(x) for x in args.tiling.split(","))
        prob.set_tiling(smcx.KIND_LOGL, S, chunk, so)
        tuned = (S, chunk, so, float("nan"))
    else:
        tuned = prob.autotune(smcx.KIND_LOGL, off, th, None, reps=2)
    outs = tuple(torch.empty(n, dtype=torch.float64, device=dev) for n in (w.N, w.N, w.N, 3))

    def step():
        smcx.reweight_extend(prob, T1, T2, off, th, 1.0, out=outs)

    ms, kern_ms, _ = timed(step, prob, args.steps, args.warmup)
    value = w.N / (ms * 1e-3)
    log(f"[bench] reweight {ms:.3f} ms/step, segment kernel {kern_ms:.3f} ms")
    rl = roofline(w.model, "fwd", component_samples(w, T1, T2), kern_ms,
                  "pop_kernel (segment forward)")
    cpu = accuracy = None
    if not args.no_cpu_baseline:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import parity as pm
        oracle.build(force=False)
        d_host = d.cpu().numpy()
        rng = np.random.default_rng(2025)
        idx, sub = cpu_sample(w, lambda s: oracle.reweight_extend(w.model, d_host, w.t_start, w.dt,
                                                                  w.sigma, T1, T2, s.offsets,
                                                                  s.theta, 1.0),
                              args.cpu_seconds, rng)
        t0 = time.perf_counter()
        ref = oracle.reweight_extend(w.model, d_host, w.t_start, w.dt, w.sigma, T1, T2, sub.offsets,
                                     sub.theta, 1.0)[0]
        cpu_s = time.perf_counter() - t0
        cpu = {"value": len(idx) / cpu_s, "unit": "evals/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"{len(idx)} of {w.N} particles, samples [{T1}, {T2}), {cpu_s:.1f} s"}
        el = pm.logl_errors(outs[0].cpu().numpy()[idx], ref)
        accuracy = {"checked_particles": len(idx), "logl_ext_max_rel_err": float(el.max())}
    sc = outs[3].cpu().numpy()
    return dict(metric="particle segment-logL evals/sec for data-assimilation reweighting",
                value=value, unit="evals/s", ms_per_step=ms,
                config={"workload": w.name, "T1": T1, "T2": T2, "N": w.N, "M": w.M,
                        "K": f"U{{0..{w.k_max}}}",
                        "tiling": {"S": tuned[0], "chunk_len": tuned[1], "sorted": tuned[2]},
                        "ESS_at_delta_beta_1": float(sc[0])},
                accuracy=accuracy, roofline=rl, cpu_baseline=cpu)


def bench_mutate(args, w, dev, smcx, np, torch):
    from paper_2609_17674_amd import workloads as wl
    d, prob, off, th0 = setup(w, dev, smcx, torch)
    beta = torch.tensor(w.beta, device=dev)
    D, eps = int(w.extra["max_depth"]), float(w.extra["eps"])
    if args.tiling:
        S, chunk, so = (int(x) for x in args.tiling.split(","))
        prob.set_tiling(smcx.KIND_GRAD, S, chunk, so)
    else:
        prob.autotune(smcx.KIND_GRAD, off, th0, beta, reps=3)
        prob.autotune(smcx.KIND_DELTA, off, th0, beta, reps=3)
    smcx.nuts_reserve(prob, D)
    mom, dirs, ul, ut = wl.nuts_draws(w.N, w.M, w.P, D, seed=4242)
    mom, dirs, ul, ut = (torch.tensor(x, device=dev) for x in (mom, dirs, ul, ut))
    lo = torch.tensor(wl.PULSE_PRIOR[:, 0].copy(), device=dev)
    hi = torch.tensor(wl.PULSE_PRIOR[:, 1].copy(), device=dev)
    tb = torch.tensor(w.extra["theta_birth"], device=dev)
    di = torch.tensor(w.extra["death_idx"], device=dev)
    l0, g0 = smcx.logl_grad_batch(prob, off, th0, beta)
    q, l, g = th0.clone(), l0.clone(), g0.clone()
    state = {}

    def step():
        q.copy_(th0)
        l.copy_(l0)
        g.copy_(g0)
        state["out"] = smcx.nuts_transition(prob, off, beta, eps, D, q, l, g, mom, dirs, ul, ut,
                                            lo, hi)
        state["delta"] = smcx.delta_logl_birth_death(prob, off, q, beta, tb, di)

    ms, kern_ms, kern_n = timed(step, prob, args.steps, args.warmup)
    depth, steps, status = (x.cpu().numpy() for x in state["out"])
    total_steps = int(steps.sum())
    value = total_steps / (ms * 1e-3)
    log(f"[bench] NUTS+RJ {ms:.3f} ms/step, {total_steps} leapfrog grads, {value:.3e} grads/s")
    return dict(metric="leapfrog gradient evals/sec inside batched NUTS (ragged trajectories)",
                value=value, unit="evals/s", ms_per_step=ms,
                config={"workload": w.name, "T": w.T, "N": w.N, "M": w.M, "max_depth": D,
                        "eps": eps, "beta": 0.5,
                        "depth_histogram": np.bincount(depth, minlength=D + 1).tolist(),
                        "status_counts": np.bincount(status, minlength=4).tolist(),
                        "leapfrog_steps": total_steps,
                        "delta_pass_ms": kern_ms})


def bench_smc(args, w, dev, smcx, np, torch):
    """Whole SMC runs on the pulse problem at the paper's pulse settings
    (Sec. "Sequence of gaussian pulses": N = 6000, K in [1, 10], alpha = 0.9,
    p_NUTS / p_birth / p_death = 0.6 / 0.2 / 0.2) with NUTS on the Gauss-Newton
    mass matrix (Sec. "No-U-Turn-Sampler"): timed prior-start runs on all
    samples, then a posterior-start run from a population sampled on the first
    half (that preparatory run is not timed). One prior-start run with the
    identity mass matrix is reported beside them."""
    from paper_2609_17674_amd import smc
    from paper_2609_17674_amd import workloads as wl
    d = torch.tensor(w.noise, device=dev) + smcx.template_sum(w.model, torch.tensor(w.inj, device=dev),
                                                               w.T, w.t_start, w.dt)
    N, k_hi = w.N, w.k_max
    lo = torch.tensor(wl.PULSE_PRIOR[:, 0].copy(), device=dev)
    hi = torch.tensor(wl.PULSE_PRIOR[:, 1].copy(), device=dev)
    prob = smcx.Problem(w.model, d, w.t_start, w.dt, w.sigma, k_hi, N, N * k_hi)
    for kind in (smcx.KIND_GRAD, smcx.KIND_LOGL):
        prob.set_tiling(kind, 32, 4096, 1)
    prob.set_tiling(smcx.KIND_DELTA, 16, 4096, 1)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    runs = []
    for r in range(args.warmup + args.steps):
        cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=300, seed=100 + r, metric=True)
        res, t = timed(lambda: smc.run_prior_start(prob, lo, hi, cfg))
        log(f"[bench] prior-start run {r}: {res.iterations} iterations, {t:.2f} s, "
            f"K histogram {res.k_hist[-1]}, log Z {res.log_evidence:.2f}")
        if r >= args.warmup:
            runs.append((t, res))
    ms = 1e3 * sum(t for t, _ in runs) / len(runs)
    iters = [res.iterations for _, res in runs]
    grads = sum(sum(res.nuts_steps) for _, res in runs)
    ident, t_ident = timed(lambda: smc.run_prior_start(
        prob, lo, hi, smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=300, seed=100)))
    log(f"[bench] identity-metric prior-start: {ident.iterations} iterations, {t_ident:.2f} s, "
        f"K histogram {ident.k_hist[-1]}, log Z {ident.log_evidence:.2f}")
    half = w.T // 2
    p1 = smcx.Problem(w.model, d[:half].contiguous(), w.t_start, w.dt, w.sigma, k_hi, N, N * k_hi)
    first = smc.run_prior_start(p1, lo, hi, smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=300,
                                                           seed=7, metric=True))
    cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=300, seed=8, metric=True)
    post, t_post = timed(lambda: smc.run_posterior_start(prob, half, first.offsets, first.theta,
                                                         lo, hi, cfg))
    log(f"[bench] posterior-start: {post.iterations} iterations, {t_post:.2f} s")
    value = N * sum(iters) / (sum(t for t, _ in runs))
    return dict(metric="particle-iterations/sec of whole prior-start SMC runs (pulse problem)",
                value=value, unit="particle-iterations/s", ms_per_step=ms,
                config={"workload": "smc_pulses", "T": w.T, "N": N, "n_injected": len(w.inj),
                        "K_range": [1, k_hi], "alpha": 0.9, "p_moves": [0.6, 0.2, 0.2],
                        "n_mutations": 4, "nuts_max_depth": 6,
                        "nuts_mass_matrix": "per-source Gauss-Newton block averaged over the "
                                            "population once per mutation step, + prior "
                                            "precision; eps 0.3 whitened",
                        "prior_start": {"iterations": iters, "seconds": [round(t, 3) for t, _ in runs],
                                        "final_K_hist": runs[-1][1].k_hist[-1],
                                        "log_evidence": [round(r.log_evidence, 2) for _, r in runs],
                                        "leapfrog_grads_per_s": grads / sum(t for t, _ in runs)},
                        "prior_start_identity_metric": {
                            "iterations": ident.iterations, "seconds": round(t_ident, 3),
                            "final_K_hist": ident.k_hist[-1],
                            "log_evidence": round(ident.log_evidence, 2)},
                        "posterior_start": {"split": half, "iterations": post.iterations,
                                            "seconds": round(t_post, 3),
                                            "final_K_hist": post.k_hist[-1]}})


def bench_metric(args, w, dev, smcx, np, torch):
    """Gauss-Newton metric of every particle of the headline population on the
    matrix cores: one smcx_gauss_newton_metric call per step."""
    d, prob, off, th = setup(w, dev, smcx, torch)
    beta = torch.tensor(w.beta, device=dev)
    fo = smcx.metric_offsets(prob, off)
    F = torch.empty(int(fo[-1]), dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def step():
        smcx.gauss_newton_metric(prob, off, th, beta, f_offsets=fo, out=F)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.steps
    prob.device_status()
    K = np.diff(w.offsets)
    n = K * w.P
    nb = 1 if w.k_max * w.P <= 32 else (2 if w.k_max * w.P <= 64 else 4)
    useful = float(np.sum(n.astype(np.float64) ** 2) * w.T * 2)        # sum_i n_i^2 T (FMA = 2)
    issued = float(np.count_nonzero(K) * (w.T / 8) * nb * (nb + 1) / 2 * 2 * 32 * 32 * 8)
    jvals = float(np.count_nonzero(K) * 32 * nb * w.T)                  # J~ entries formed
    tf = issued / (ms * 1e-3) / 1e12
    value = w.N / (ms * 1e-3)
    # the J entries are synthesised on the vector units, 8 FP32-FMA slots each
    # (sub 1/2, fma 1, mul 1/2, exp2 2, two fma 2, mul 1/2, f16 convert 1,
    # select 1/2), which is what bounds the kernel; the matrix cores carry the
    # contraction
    slots_tf = 2.0 * 8 * jvals / (ms * 1e-3) / 1e12
    log(f"[bench] metric {ms:.4f} ms/step, {value:.4e} particles/s, MFMA {tf:.1f} TFLOP/s issued")
    return dict(metric="particle Gauss-Newton metrics/sec (FP16 matrix cores, FP64 output)",
                value=value, unit="particles/s", ms_per_step=ms,
                config={"workload": "metric_pulse_batch", "T": w.T, "N": w.N, "M": w.M,
                        "K": f"U{{0..{w.k_max}}}", "coordinate_blocks": nb},
                roofline={"bound": "alu", "achieved": round(slots_tf, 3), "peak": PEAK_FP32_TFLOPS,
                          "unit": "TFLOP/s", "frac": round(slots_tf / PEAK_FP32_TFLOPS, 4),
                          "traffic": None, "kernel": "metric_kernel", "kernel_ms": round(ms, 5),
                          "work": f"{jvals:.4e} J entries x 8 FP32-FMA slots x 2 flops",
                          "mfma_issued_tflops": round(tf, 2), "mfma_peak_fp16_tflops": 2500.0,
                          "mfma_frac": round(tf / 2500.0, 4),
                          "useful_tflops": round(useful / (ms * 1e-3) / 1e12, 2)})


# FP64 operations per lane of the wave per source in one logL + gradient
# evaluation of the frequency-domain model: envelope synthesis 175 (two
# detector-tensor products per channel, retarded time, phase, sincospi),
# forward FFT 60, placement 8, inverse FFT 60, envelope again 175, the eight
# derivatives and their products with the inverse FFT 390, reductions 48.
GBLISA_FLOPS_PER_LANE = 920
PEAK_FP64_TFLOPS = 78.6


def bench_gblisa(args, dev, smcx, np, torch):
    """LISA Galactic binaries in the frequency domain at the paper's settings
    (Sec. "LISA Galactic binaries": one year, ten sources with f0 on a grid in
    [0.9998, 1.0006] mHz, noise-free A and E data, N = 40000 particles, K in
    [1, 10]); one logl_grad_batch call per step, beta ~ U[0, 1]."""
    from paper_2609_17674_amd import workloads as wl
    w = wl.make_gblisa(N=40000, k_lo=1, k_hi=10, n_inj=10, beta="uniform", noise=False)
    log(f"[bench] workload gb_lisa: N={w.N} M={w.M} B={w.B} bins")
    inj = torch.tensor(w.inj, device=dev)
    d = smcx.template_spectrum(wl.GBLISA, inj, w.T_obs, w.k0, w.B)
    prob = smcx.Problem.frequency_domain(wl.GBLISA, d, w.k0, w.T_obs, w.S, w.k_max, w.N, w.M)
    off, th = torch.tensor(w.offsets, device=dev), torch.tensor(w.theta, device=dev)
    beta = torch.tensor(w.beta, device=dev)
    logl = torch.empty(w.N, dtype=torch.float64, device=dev)
    grad = torch.empty_like(th)

    def step():
        smcx.logl_grad_batch(prob, off, th, beta, logl=logl, grad=grad)

    ms, kern_ms, _ = timed(step, prob, args.steps, args.warmup)
    value = w.N / (ms * 1e-3)
    log(f"[bench] {ms:.4f} ms/step, kernel {kern_ms:.4f} ms, {value:.4e} evals/s")
    flops = float(w.M) * 64 * GBLISA_FLOPS_PER_LANE
    achieved = flops / (kern_ms * 1e-3) / 1e12
    rl = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
          "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
          "kernel": "fd_kernel (fused forward+adjoint, FP64)", "kernel_ms": round(kern_ms, 5),
          "work": f"{w.M} sources x 64 lanes x {GBLISA_FLOPS_PER_LANE} FP64 flops"}
    cpu = accuracy = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        d_host = d.cpu().numpy()
        rng = np.random.default_rng(2025)

        def orc_eval(s):
            return oracle.gblisa_logl_grad(d_host, w.k0, w.T_obs, w.S, s.offsets, s.theta, s.beta)

        probe = np.sort(rng.choice(w.N, size=32, replace=False))
        sub = _gb_subset(w, probe)
        t0 = time.perf_counter()
        orc_eval(sub)
        per = (time.perf_counter() - t0) / len(probe)
        n = int(min(w.N, max(64, args.cpu_seconds / max(per, 1e-9))))
        idx = np.sort(rng.choice(w.N, size=n, replace=False))
        sub = _gb_subset(w, idx)
        t0 = time.perf_counter()
        ref_l, ref_g = orc_eval(sub)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": n / cpu_s, "unit": "evals/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"{n} of {w.N} particles of the same workload (seeded), all {w.B} bins, "
                         f"{cpu_s:.1f} s"}
        log(f"[bench] cpu oracle {n} particles in {cpu_s:.1f} s")
        out_l, out_g = logl.cpu().numpy(), grad.cpu().numpy()
        rows = np.concatenate([np.arange(w.offsets[i], w.offsets[i + 1]) for i in idx])
        el = np.abs(out_l[idx] - ref_l) / np.abs(ref_l)
        nat = np.array([w.T_obs, w.T_obs ** 2, 1, 1, 1, 1, 1, 1])
        gr = []
        for j, i in enumerate(idx):
            a, b = sub.offsets[j], sub.offsets[j + 1]
            gg, rr = out_g[rows[a:b]] / nat, ref_g[a:b] / nat
            gr.append(np.linalg.norm(gg - rr) / max(np.linalg.norm(rr), 1e-300))
        accuracy = {"checked_particles": n, "logl_max_rel_err": float(el.max()),
                    "grad_max_rel_err": float(max(gr))}
    return dict(metric="particle logL+grad evals/sec, LISA Galactic binaries (frequency domain, "
                       "A+E, FP64)",
                value=value, unit="evals/s", ms_per_step=ms,
                config={"workload": "gb_lisa", "T_obs_s": w.T_obs, "bins": w.B, "N": w.N,
                        "M": w.M, "K": f"U{{1..{w.k_max}}}", "beta": "U[0,1]",
                        "n_injected": len(w.inj), "data": "noise-free"},
                accuracy=accuracy, roofline=rl, cpu_baseline=cpu, dtype="f64")


def bench_smc_gblisa(args, dev, smcx, np, torch):
    """Whole prior-start SMC runs on the Galactic-binary problem at the paper's
    settings (Sec. "LISA Galactic binaries": one year, ten noise-free
    binaries, N = 40000 particles, K in [1, 10], alpha = 0.9, moves 0.6 / 0.2
    / 0.2) with NUTS on the per-source Gauss-Newton mass matrix."""
    from paper_2609_17674_amd import smc
    from paper_2609_17674_amd import workloads as wl
    N, k_hi = 40000, 10
    w = wl.make_gblisa(N=16, k_lo=1, k_hi=k_hi, n_inj=10, noise=False)
    inj = torch.tensor(w.inj, device=dev)
    d = smcx.template_spectrum(wl.GBLISA, inj, w.T_obs, w.k0, w.B)
    prob = smcx.Problem.frequency_domain(wl.GBLISA, d, w.k0, w.T_obs, w.S, k_hi, N, N * k_hi)
    lo = torch.tensor(wl.GBLISA_PRIOR[:, 0].copy(), device=dev)
    hi = torch.tensor(wl.GBLISA_PRIOR[:, 1].copy(), device=dev)
    runs = []
    for r in range(args.warmup + args.steps):
        cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=400, seed=300 + r, metric=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = smc.run_prior_start(prob, lo, hi, cfg)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        log(f"[bench] GB prior-start run {r}: {res.iterations} iterations, {t:.2f} s, "
            f"K histogram {res.k_hist[-1]}, log Z {res.log_evidence:.1f}")
        if r >= args.warmup:
            runs.append((t, res))
    iters = [res.iterations for _, res in runs]
    total = sum(t for t, _ in runs)
    grads = sum(sum(res.nuts_steps) for _, res in runs)
    return dict(metric="particle-iterations/sec of whole prior-start SMC runs (LISA Galactic "
                       "binaries, frequency domain)",
                value=N * sum(iters) / total, unit="particle-iterations/s",
                ms_per_step=1e3 * total / len(runs), dtype="f64",
                config={"workload": "smc_gblisa", "T_obs_s": w.T_obs, "bins": w.B, "N": N,
                        "n_injected": 10, "K_range": [1, k_hi], "alpha": 0.9,
                        "p_moves": [0.6, 0.2, 0.2], "n_mutations": 4, "nuts_max_depth": 6,
                        "nuts_mass_matrix": "per-source Gauss-Newton block averaged over the "
                                            "population once per mutation step, + prior "
                                            "precision; eps 0.3 whitened",
                        "iterations": iters, "seconds": [round(t, 3) for t, _ in runs],
                        "final_K_hist": runs[-1][1].k_hist[-1],
                        "log_evidence": [round(r.log_evidence, 2) for _, r in runs],
                        "leapfrog_grads_per_s": grads / total})


def _gb_subset(w, idx):
    import numpy as np
    from types import SimpleNamespace
    K = w.K[idx]
    off = np.zeros(len(idx) + 1, dtype=np.int64)
    off[1:] = np.cumsum(K)
    rows = np.concatenate([np.arange(w.offsets[i], w.offsets[i + 1]) for i in idx])
    return SimpleNamespace(offsets=off, theta=w.theta[rows], beta=w.beta[idx])


def issue_probe(args, smcx, torch):
    """VALU issue ceilings of this device: each instruction kind of the
    population kernels at 1, 2, 4 and 8 waves per SIMD, in lane-instructions
    per clock per compute unit (published engine clock 2.4 GHz)."""
    props = torch.cuda.get_device_properties(0)
    n_cu = props.multi_processor_count
    inp = torch.rand(256, dtype=torch.float32, device="cuda")
    out = torch.empty(n_cu * 8 * 256, dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    table = {}
    for kind in smcx.PROBE_KINDS:
        row = {}
        for wps in (1, 2, 4, 8):
            blocks, iters = n_cu * wps, 2048
            smcx.issue_probe(kind, blocks, 16, inp, out)
            best = float("inf")
            for _ in range(max(args.steps, 1)):
                ev[0].record()
                ops = smcx.issue_probe(kind, blocks, iters, inp, out)
                ev[1].record()
                torch.cuda.synchronize()
                best = min(best, ev[0].elapsed_time(ev[1]))
            row[wps] = round(ops / (best * 1e-3) / n_cu / CLOCK_HZ, 2)
        table[kind] = row
        log(f"[bench] {kind}: lanes/clk/CU by waves per SIMD {row}")
    print(json.dumps({"issue_probe_lanes_per_clk_per_cu": table, "compute_units": n_cu,
                      "clock_hz": CLOCK_HZ}), flush=True)


def copy_probe(args, torch):
    """Device-to-device copy of a known size, for calibrating HBM byte counters."""
    n = 1 << 26  # 64 Mi float32 = 256 MiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(max(args.steps, 1)):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_launch": 4 * n,
                      "copy_probe_bytes_written_per_launch": 4 * n, "launches": args.steps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="gb_grad",
                    choices=["gb_grad", "pulse_batch", "gb_extend", "pulse_mutate", "smc_pulses",
                             "metric", "gb_lisa", "smc_gblisa", "copy_probe", "issue_probe"])
    ap.add_argument("--tiling", default="",
                    help="S,chunk_len,sorted: fixed tiling of the timed call kind, no autotuning")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu1-seconds", type=float, default=3.0,
                    help="budget of the one-thread oracle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="gb_grad only: skip the pulse_batch line attached as 'secondary'")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU only (N=1); runs on several GPUs are not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_17674_amd import smcx
    from paper_2609_17674_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "copy_probe":
        copy_probe(args, torch)
        return
    if args.workload == "issue_probe":
        issue_probe(args, smcx, torch)
        return
    secondary = None
    if args.workload == "gb_lisa":
        res = bench_gblisa(args, dev, smcx, np, torch)
    elif args.workload == "smc_gblisa":
        res = bench_smc_gblisa(args, dev, smcx, np, torch)
    elif args.workload == "smc_pulses":
        w = wl.make_config("pulse_batch", N=6000, n_inj=10, k_lo=1, k_hi=10)
        res = bench_smc(args, w, dev, smcx, np, torch)
    elif args.workload == "metric":
        res = bench_metric(args, wl.make_config("pulse_batch"), dev, smcx, np, torch)
    else:
        w = wl.make_config(args.workload)
        log(f"[bench] workload {w.name}: N={w.N} T={w.T} M={w.M}")
        if args.workload in ("pulse_batch", "gb_grad"):
            res = bench_grad(args, w, dev, smcx, np, torch, args.cpu_seconds, args.cpu1_seconds,
                             check_all=args.workload == "pulse_batch")
            if args.workload == "gb_grad" and not args.no_secondary:
                w2 = wl.make_config("pulse_batch")
                log(f"[bench] secondary workload {w2.name}: N={w2.N} T={w2.T} M={w2.M}")
                r2 = bench_grad(args, w2, dev, smcx, np, torch, args.cpu_seconds,
                                args.cpu1_seconds, check_all=True)
                secondary = {k: r2[k] for k in ("value", "unit", "ms_per_step", "config",
                                                "plain_gpu", "speedup_vs_plain", "accuracy",
                                                "roofline", "cpu_baseline")}
        elif args.workload == "gb_extend":
            res = bench_extend(args, w, dev, smcx, np, torch)
        else:
            res = bench_mutate(args, w, dev, smcx, np, torch)
    line = {
        "metric": res["metric"],
        "value": res["value"],
        "unit": res["unit"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res.get("dtype", "f32+f64"),
        "data": "synthetic",
        "config": res["config"],
    }
    for key in ("plain_gpu", "speedup_vs_plain", "accuracy", "roofline", "cpu_baseline"):
        if key in res:
            line[key] = res[key]
    if secondary is not None:
        line["secondary"] = secondary
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
