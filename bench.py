#!/usr/bin/env python3
"""Throughput of the batched fused log-likelihood + gradient on one MI355X.

A step is one logl_grad_batch call over the whole population of the
workload (template synthesis, residual, FP64 inner products, adjoint
gradient and ragged batching in one pass): the unit of work is one particle
log-likelihood + gradient evaluation. The same population is then run
through the plain one-particle-per-launch FP64 form on the same GPU, and
through the FP64 CPU oracle on a bounded sample on the host cores; the
oracle's results on that sample also give the reported error of the GPU
path. Inputs are seeded synthetic workloads resident in device memory
before the timed region starts.

Prints one JSON line. Usage: python bench.py [--steps K] [--warmup W]
[--workload pulse_batch|gb_grad] [--gpus 1].
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle logL+grad evals/sec (ragged K) vs plain GPU form at ≤1e-6 rel err"

# MI355X published peaks: 256 CUs at 2.4 GHz, FP32 vector 157.3 TFLOP/s
# (128 FP32 FMA lanes per CU per clock), FP64 vector 78.6 TFLOP/s.
PEAK_FP32_TFLOPS = 157.3

# Issue cost of one component-sample of the fused forward + adjoint pass in
# FP32-FMA-equivalent VALU slots (FP32 op = 1, FP64 op = 2, transcendental =
# 4; the weights are the published FP32:FP64 ratio and the measured
# exp/sin/cos issue rate on gfx950). Pulse: forward add, fma, mul, exp2,
# fma; adjoint add, fma, mul, exp2, mul, add, mul, add, fma. Sinusoid:
# forward 2 FP64 fma, cvt, mul, sin, fma; adjoint 2 FP64 fma, cvt, mul,
# sin, cos, fma, mul, add, fma, fma.
SLOTS_PER_COMPONENT_SAMPLE = {0: 8 + 12, 1: 11 + 19}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="pulse_batch", choices=["pulse_batch", "gb_grad"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (N=1); multi-GPU runs are not part of "
              "it", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_17674_amd import smcx
    from paper_2609_17674_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = wl.make_config(args.workload)
    log(f"[bench] workload {w.name}: N={w.N} T={w.T} M={w.M}")
    inj = torch.tensor(w.inj, device=dev)
    d = torch.tensor(w.noise, device=dev) + smcx.template_sum(w.model, inj, w.T, w.t_start, w.dt)
    prob = smcx.Problem(w.model, d, w.t_start, w.dt, w.sigma, w.k_max, w.N, w.M)
    off = torch.tensor(w.offsets, device=dev)
    th = torch.tensor(w.theta, device=dev)
    beta = torch.tensor(w.beta, device=dev)
    logl = torch.empty(w.N, dtype=torch.float64, device=dev)
    grad = torch.empty_like(th)

    tuned = prob.autotune(smcx.KIND_GRAD, off, th, beta, reps=5)
    log(f"[bench] autotuned tiling S={tuned[0]} chunk={tuned[1]} sorted={tuned[2]} "
        f"({tuned[3]:.4f} ms/call)")

    def step():
        smcx.logl_grad_batch(prob, off, th, beta, logl=logl, grad=grad)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prob.device_status()
    log(f"[bench] warmup done ({args.warmup} steps)")

    prob.profile_begin(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, kern_n = prob.profile_end()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = w.N / (ms_per_step * 1e-3)
    kern_avg_ms = kern_ms / max(kern_n, 1)
    log(f"[bench] {ms_per_step:.4f} ms/step, kernel {kern_avg_ms:.4f} ms, {value:.4e} evals/s")

    comp_samples = float(w.M) * w.T
    slots = SLOTS_PER_COMPONENT_SAMPLE[w.model] * comp_samples
    achieved = 2.0 * slots / (kern_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                "kernel": "pop_kernel (fused forward+adjoint)",
                "kernel_ms": round(kern_avg_ms, 5),
                "work": f"{comp_samples:.4e} component-samples x "
                        f"{SLOTS_PER_COMPONENT_SAMPLE[w.model]} FP32-FMA-equivalent slots"}

    out_l = logl.cpu().numpy()
    out_g = grad.cpu().numpy()

    plain = None
    if not args.no_plain:
        pl = torch.empty_like(logl)
        pg = torch.empty_like(grad)
        sub = min(64, w.N)
        msub = int(w.offsets[sub])
        smcx.plain_logl_grad(prob, w.offsets[:sub + 1], th[:msub], beta[:sub],
                             logl=pl[:sub], grad=pg[:msub])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smcx.plain_logl_grad(prob, w.offsets, th, beta, logl=pl, grad=pg)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain_ms = (t1 - t0) * 1e3
        plain = {"value": w.N / (plain_ms * 1e-3), "unit": "evals/s", "ms_per_step": plain_ms,
                 "form": "one particle per forward+adjoint launch pair, FP64"}
        plain_l, plain_g = pl.cpu().numpy(), pg.cpu().numpy()
        log(f"[bench] plain form {plain_ms:.1f} ms/step")

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        d_host = d.cpu().numpy()
        rng = np.random.default_rng(2024)
        probe = wl.subsample(w, np.sort(rng.choice(w.N, size=min(32, w.N), replace=False)))
        t0 = time.perf_counter()
        oracle.logl_grad(w.model, d_host, w.t_start, w.dt, w.sigma, probe.offsets, probe.theta,
                         probe.beta)
        per = (time.perf_counter() - t0) / probe.N
        n = int(min(w.N, max(64, args.cpu_seconds / max(per, 1e-9))))
        idx = np.sort(rng.choice(w.N, size=n, replace=False))
        sub = wl.subsample(w, idx)
        t0 = time.perf_counter()
        ref_l, ref_g = oracle.logl_grad(w.model, d_host, w.t_start, w.dt, w.sigma, sub.offsets,
                                        sub.theta, sub.beta)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": n / cpu_s, "unit": "evals/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"{n} of {w.N} particles of the same workload (seeded), all {w.T} "
                         f"samples, {cpu_s:.1f} s"}
        log(f"[bench] cpu oracle {n} particles in {cpu_s:.1f} s")

        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import parity as pm
        rows = np.concatenate([np.arange(w.offsets[i], w.offsets[i + 1]) for i in idx])
        el = pm.logl_errors(out_l[idx], ref_l)
        rel, cos = pm.grad_errors(w.model, sub.offsets, sub.theta, out_g[rows], ref_g, w.T, w.dt)
        accuracy = {"checked_particles": n, "logl_max_rel_err": float(el.max()),
                    "grad_max_rel_err": float(rel.max()) if len(rel) else 0.0,
                    "grad_min_cos": float(cos.min()) if len(cos) else 1.0}
        if plain is not None:
            pel = pm.logl_errors(plain_l[idx], ref_l)
            prel, _ = pm.grad_errors(w.model, sub.offsets, sub.theta, plain_g[rows], ref_g, w.T,
                                     w.dt)
            plain["logl_max_rel_err"] = float(pel.max())
            plain["grad_max_rel_err"] = float(prel.max()) if len(prel) else 0.0

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "T": w.T, "N": w.N, "M": w.M,
                   "K": f"U{{0..{w.k_max}}}", "beta": "U[0,1]" if w.name == "pulse_batch" else "1",
                   "precision": "FP32 synthesis/residual, FP64 phase and accumulation",
                   "tiling": {"S": tuned[0], "chunk_len": tuned[1], "sorted": tuned[2]}},
        "plain_gpu": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "accuracy": accuracy,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
