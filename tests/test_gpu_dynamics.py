"""Leapfrog and NUTS on the GPU against the oracle (through the C ABI)."""
import sys

import numpy as np
import pytest
import torch

import parity as pm
from paper_2609_17674_amd import workloads as wl

pytestmark = pytest.mark.gpu
PULSE, GB = wl.PULSE, wl.GBSINE


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _setup(lib, cfg, **ov):
    w = wl.make_config(cfg, **ov)
    d = pm.data_of(w)
    prob = lib.Problem(w.model, pm.to_dev(d), w.t_start, w.dt, w.sigma, w.k_max, w.N, max(w.M, 1))
    return w, d, prob


@pytest.mark.parametrize("cfg,ov", [("pulse_mutate", dict(N=200, T=4096)),
                                    ("pulse_mutate", dict(N=60, T=9000)),
                                    ("gb_grad", dict(N=50, T=5000, k_hi=8))],
                         ids=["pulse", "pulse_chunks", "gb"])
def test_leapfrog_step_matches_oracle(lib, orc, cfg, ov):
    w, d, prob = _setup(lib, cfg, **ov)
    say("leapfrog", cfg, ov)
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(w.theta.shape)
    dirs = np.where(rng.random(w.N) < 0.5, -1, 1).astype(np.int8)
    active = (rng.random(w.N) < 0.8).astype(np.uint8)
    eps = 1e-4 if w.model == PULSE else 1e-12
    if w.model == GB:  # natural step sizes per coordinate are very different; scale momenta
        Tobs = w.T * w.dt
        p0 = p0 * np.array([1.0, 1.0 / Tobs, 1.0 / Tobs ** 2, 1.0]) * 1e6
    off, th, be = pm.to_dev(w.offsets), pm.to_dev(w.theta), pm.to_dev(w.beta)
    l0, g0 = lib.logl_grad_batch(prob, off, th, be)
    q1, p1, g1, l1 = lib.leapfrog(prob, off, be, eps, th, pm.to_dev(p0), g0, dir=pm.to_dev(dirs),
                                  active=pm.to_dev(active))
    torch.cuda.synchronize()
    prob.device_status()
    q1, p1, g1, l1 = (x.cpu().numpy() for x in (q1, p1, g1, l1))
    g0h = g0.cpu().numpy()
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        if a == b:
            continue
        if not active[i]:
            assert np.array_equal(q1[a:b], w.theta[a:b]) and np.array_equal(p1[a:b], p0[a:b])
            assert np.array_equal(g1[a:b], g0h[a:b])
            continue
        sub = np.array([0, b - a])
        e = eps * dirs[i]
        rq, rp, rl, rg = orc.leapfrog(w.model, d, w.t_start, w.dt, w.sigma, sub, w.theta[a:b], p0[a:b],
                                      w.beta[i:i + 1], e)
        _, rg0 = orc.logl_grad(w.model, d, w.t_start, w.dt, w.sigma, sub, w.theta[a:b],
                               w.beta[i:i + 1])
        pm.assert_logl(l1[i:i + 1], rl)
        pm.assert_grad(w.model, sub, rq, g1[a:b], rg, w.T, w.dt)
        # positions and momenta: the kicks carry the gradient tolerance (1e-5 of the
        # natural-coordinate norm, here doubled) into per-coordinate bounds
        s0 = pm.natural_scale(w.model, w.theta[a:b], w.T, w.dt)
        s1 = pm.natural_scale(w.model, rq, w.T, w.dt)
        dg0 = 2e-5 * np.linalg.norm(rg0 * s0) / s0
        dg1 = 2e-5 * np.linalg.norm(rg * s1) / s1
        tol_q = 0.5 * e * e * dg0 + 1e-14 * np.abs(rq)
        tol_p = 0.5 * abs(e) * (dg0 + dg1) + 1e-14 * np.abs(rp)
        assert np.all(np.abs(q1[a:b] - rq) <= tol_q), i
        assert np.all(np.abs(p1[a:b] - rp) <= tol_p), i


def test_leapfrog_reversible_on_gpu(lib, orc):
    w, d, prob = _setup(lib, "pulse_mutate", N=64, T=4096)
    say("leapfrog_reversible")
    rng = np.random.default_rng(9)
    off, be = pm.to_dev(w.offsets), pm.to_dev(np.full(w.N, 0.02))
    q = pm.to_dev(w.theta)
    p = pm.to_dev(rng.standard_normal(w.theta.shape))
    _, g = lib.logl_grad_batch(prob, off, q, be)
    q0, p0 = q.clone(), p.clone()
    for _ in range(20):
        q, p, g, _ = lib.leapfrog(prob, off, be, 2e-4, q, p, g)
    p = -p
    for _ in range(20):
        q, p, g, _ = lib.leapfrog(prob, off, be, 2e-4, q, p, g)
    torch.cuda.synchronize()
    assert torch.allclose(q, q0, rtol=0, atol=1e-9)
    assert torch.allclose(-p, p0, rtol=0, atol=1e-6)


def _nuts_inputs(lib, w, prob, D, seed, eps):
    mom, dirs, ul, ut = wl.nuts_draws(w.N, w.M, w.P, D, seed)
    dev = {k: pm.to_dev(v) for k, v in dict(mom=mom, dirs=dirs, ul=ul, ut=ut).items()}
    off, th, be = pm.to_dev(w.offsets), pm.to_dev(w.theta), pm.to_dev(w.beta)
    l0, g0 = lib.logl_grad_batch(prob, off, th, be)
    prior = wl.PULSE_PRIOR if w.model == PULSE else None
    lo = hi = None
    if prior is not None:
        lo, hi = pm.to_dev(prior[:, 0].copy()), pm.to_dev(prior[:, 1].copy())
    return (mom, dirs, ul, ut), dev, off, th, be, l0, g0, lo, hi


def test_nuts_graph_replays_equal_eager(lib, orc):
    w, d, prob = _setup(lib, "pulse_mutate", N=300, T=4096)
    say("nuts_graph")
    D = 6
    lib.nuts_reserve(prob, D)
    host, dev, off, th, be, l0, g0, lo, hi = _nuts_inputs(lib, w, prob, D, 11, 2e-4)
    results = []
    for use_graph in (False, True, True, True):
        q, l, g = th.clone(), l0.clone(), g0.clone()
        depth, steps, status = lib.nuts_transition(prob, off, be, 2e-4, D, q, l, g, dev["mom"],
                                                   dev["dirs"], dev["ul"], dev["ut"], lo, hi,
                                                   use_graph=use_graph)
        torch.cuda.synchronize()
        prob.device_status()
        results.append([x.cpu().numpy() for x in (q, l, g, depth, steps, status)])
        # eager work between graph replays
        _ = lib.logl_batch(prob, off, th, be)
        torch.cuda.synchronize()
    for r in results[1:]:
        for x, y in zip(results[0], r):
            assert np.array_equal(x, y)
    depth, steps, status = results[0][3:]
    assert np.all((status >= 0) & (status <= 3))
    has = w.K > 0
    assert np.all(status[~has] == 0) and np.all(steps[~has] == 0)
    assert np.all(steps[has] >= 1) and np.all(steps[has] <= (1 << D) - 1)
    assert np.all(steps[has] >= (1 << depth[has]) - 1)


def test_nuts_matches_oracle_statistically(lib, orc):
    w, d, prob = _setup(lib, "pulse_mutate", N=96, T=1000, k_lo=1, k_hi=4, n_inj=3)
    say("nuts_vs_oracle")
    D, eps = 6, 2e-4
    lib.nuts_reserve(prob, D)
    (mom, dirs, ul, ut), dev, off, th, be, l0, g0, lo, hi = _nuts_inputs(lib, w, prob, D, 12, eps)
    q, l, g = th.clone(), l0.clone(), g0.clone()
    depth, steps, status = lib.nuts_transition(prob, off, be, eps, D, q, l, g, dev["mom"], dev["dirs"],
                                               dev["ul"], dev["ut"], lo, hi)
    torch.cuda.synchronize()
    ref_l0, ref_g0 = orc.logl_grad(PULSE, d, w.t_start, w.dt, w.sigma, w.offsets, w.theta, w.beta)
    rq, rl, rg, rdepth, rsteps, rstatus = orc.nuts_transition(
        PULSE, d, w.t_start, w.dt, w.sigma, w.offsets, w.beta, eps, D, w.theta, ref_l0, ref_g0, mom,
        dirs, ul, ut, wl.PULSE_PRIOR[:, 0], wl.PULSE_PRIOR[:, 1])
    depth, steps, status = depth.cpu().numpy(), steps.cpu().numpy(), status.cpu().numpy()
    same = (depth == rdepth) & (status == rstatus) & (steps == rsteps)
    # FP32 vs FP64 dynamics can flip a marginal decision; most particles must agree exactly
    assert same.mean() >= 0.9, same.mean()
    qn = q.cpu().numpy()
    close = []
    for i in np.nonzero(same)[0]:
        a, b = w.offsets[i], w.offsets[i + 1]
        # same tree => (almost always) the same proposal leaf, equal up to FP32 template error
        close.append(np.allclose(qn[a:b], rq[a:b], rtol=1e-6, atol=1e-9))
    assert np.mean(close) >= 0.95, np.mean(close)
    hist = np.bincount(depth, minlength=D + 1)
    rhist = np.bincount(rdepth, minlength=D + 1)
    assert np.abs(hist - rhist).sum() <= 0.2 * w.N


def test_nuts_at_the_mutation_workload_shape(lib, orc):
    """The C4 mutation step's data and settings (T = 4096 samples, eight
    injected pulses, beta = 0.5, depth <= 8) with particles near the posterior
    (each a random subset of the injected pulses, slightly perturbed) and a
    step of 1.5e-4, so that trees grow up to the maximum depth instead of
    diverging at the first leaves as prior draws do: the GPU transition
    against the oracle's on the same draws, statistically as above."""
    w = wl.make_config("pulse_mutate", N=4)
    d = pm.data_of(w)
    rng = np.random.default_rng(5)
    N, D, eps = 160, 8, 1.5e-4
    K = rng.integers(1, len(w.inj) + 1, N)
    rows = [w.inj[rng.choice(len(w.inj), k, replace=False)]
            * (1 + rng.standard_normal((k, 3)) * np.array([2e-3, 2e-4, 2e-3])) for k in K]
    theta = np.concatenate(rows)
    offsets = wl.counts_to_offsets(K)
    beta = np.full(N, 0.5)
    say("nuts_c4_shape", N, w.T, len(theta))
    prob = lib.Problem(PULSE, pm.to_dev(d), w.t_start, w.dt, w.sigma, int(K.max()), N, len(theta))
    lib.nuts_reserve(prob, D)
    mom, dirs, ul, ut = wl.nuts_draws(N, len(theta), 3, D, 13)
    dev = {k: pm.to_dev(v) for k, v in dict(mom=mom, dirs=dirs, ul=ul, ut=ut).items()}
    off, th, be = pm.to_dev(offsets), pm.to_dev(theta), pm.to_dev(beta)
    lo, hi = pm.to_dev(wl.PULSE_PRIOR[:, 0].copy()), pm.to_dev(wl.PULSE_PRIOR[:, 1].copy())
    l0, g0 = lib.logl_grad_batch(prob, off, th, be)
    q, l, g = th.clone(), l0.clone(), g0.clone()
    depth, steps, status = lib.nuts_transition(prob, off, be, eps, D, q, l, g, dev["mom"], dev["dirs"],
                                               dev["ul"], dev["ut"], lo, hi)
    torch.cuda.synchronize()
    prob.device_status()
    ref_l0, ref_g0 = orc.logl_grad(PULSE, d, w.t_start, w.dt, w.sigma, offsets, theta, beta)
    rq, rl, rg, rdepth, rsteps, rstatus = orc.nuts_transition(
        PULSE, d, w.t_start, w.dt, w.sigma, offsets, beta, eps, D, theta, ref_l0, ref_g0, mom, dirs,
        ul, ut, wl.PULSE_PRIOR[:, 0], wl.PULSE_PRIOR[:, 1])
    depth, steps, status = depth.cpu().numpy(), steps.cpu().numpy(), status.cpu().numpy()
    same = (depth == rdepth) & (status == rstatus) & (steps == rsteps)
    print(f"[nuts] depth histogram GPU {np.bincount(depth, minlength=D + 1).tolist()}, oracle "
          f"{np.bincount(rdepth, minlength=D + 1).tolist()}; same tree {same.mean():.3f}", flush=True)
    assert np.mean(rdepth >= 3) >= 0.3, np.bincount(rdepth, minlength=D + 1)
    assert same.mean() >= 0.85, same.mean()
    assert np.mean(depth[same] >= 3) >= 0.3
    qn = q.cpu().numpy()
    close = [np.allclose(qn[offsets[i]:offsets[i + 1]], rq[offsets[i]:offsets[i + 1]],
                         rtol=1e-5, atol=1e-8) for i in np.nonzero(same)[0]]
    assert np.mean(close) >= 0.9, np.mean(close)
    hist = np.bincount(depth, minlength=D + 1)
    rhist = np.bincount(rdepth, minlength=D + 1)
    assert np.abs(hist - rhist).sum() <= 0.2 * N
