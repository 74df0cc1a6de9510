"""The prior-start SMC driver end to end on a synthetic pulse problem.

The SMC loop as a whole is parity unpinned: the paper prints no values for
it, and its components are pinned one by one elsewhere. This test checks the
qualitative behaviour the paper reports for its pulse example (Sec. "Sequence
of gaussian pulses"): the temperature reaches one, the number of components
starts spread over the prior range, and at beta = 1 the posterior over K
peaks at the injected count.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2609_17674_amd import smc
from paper_2609_17674_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_prior_start_smc_recovers_the_number_of_pulses(lib, orc):
    T = 1000
    dt = 1.0 / (T - 1)
    inj = np.array([[5.0, 0.25, 0.02], [4.0, 0.52, 0.03], [5.5, 0.76, 0.015]])
    rng = np.random.default_rng(31)
    d = rng.standard_normal(T) + orc.template_sum(wl.PULSE, inj, T, 0.0, dt)
    N, k_hi = 2048, 6
    prob = lib.Problem(wl.PULSE, torch.tensor(d, device="cuda"), 0.0, dt, 1.0, k_hi, N, N * k_hi)
    lo = torch.tensor(wl.PULSE_PRIOR[:, 0].copy(), device="cuda")
    hi = torch.tensor(wl.PULSE_PRIOR[:, 1].copy(), device="cuda")
    cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, n_mutations=4, max_depth=6, max_iters=150, seed=5)

    def report(it, info):
        print(f"[smc] it={it} beta={info['beta']:.4g} ess={info['ess']:.1f} "
              f"k={info['k_hist']} rj={info['rj_accept']:.3f} nuts_steps={info['nuts_steps']}",
              flush=True)

    print("[case] prior_start_smc", flush=True)
    sys.stdout.flush()
    res = smc.run_prior_start(prob, lo, hi, cfg, on_iteration=report)
    assert res.betas[-1] == 1.0
    assert all(b2 > b1 for b1, b2 in zip(res.betas, res.betas[1:]))
    assert np.isfinite(res.log_evidence)
    first = np.array(res.k_hist[0][1:], dtype=float) / N
    assert first.min() > 0.08  # still close to the uniform prior over K = 1..6
    final = np.array(res.k_hist[-1], dtype=float) / N
    assert int(np.argmax(final)) == 3, final
    assert final[3] >= 0.5, final
    # every particle's rows stay inside the prior box
    th = res.theta.cpu().numpy()
    assert np.all(th >= wl.PULSE_PRIOR[:, 0]) and np.all(th <= wl.PULSE_PRIOR[:, 1])


def test_posterior_start_reuses_the_shorter_run(lib, orc):
    """Sec. "Algorithm and implementation", posterior-start mode: a population
    sampled on the first half of the data is carried to the full data by the
    bridge of eq. reuse_bridge. It must end with the full data's component
    count and take fewer SMC iterations than a prior-start run on the full
    data (the trend the paper reports for its pulse example)."""
    T, split = 1000, 500
    dt = 1.0 / (T - 1)
    inj = np.array([[5.0, 0.2, 0.02], [4.0, 0.36, 0.03], [5.5, 0.75, 0.015]])
    rng = np.random.default_rng(33)
    d = rng.standard_normal(T) + orc.template_sum(wl.PULSE, inj, T, 0.0, dt)
    N, k_hi = 2048, 6
    dev = "cuda"
    lo = torch.tensor(wl.PULSE_PRIOR[:, 0].copy(), device=dev)
    hi = torch.tensor(wl.PULSE_PRIOR[:, 1].copy(), device=dev)

    def report(tag):
        def f(it, info):
            print(f"[smc {tag}] it={it} beta={info['beta']:.4g} k={info['k_hist']} "
                  f"rj={info['rj_accept']:.3f}", flush=True)
        return f

    print("[case] posterior_start", flush=True)
    p1 = lib.Problem(wl.PULSE, torch.tensor(d[:split], device=dev), 0.0, dt, 1.0, k_hi, N, N * k_hi)
    cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=150, seed=7)
    first = smc.run_prior_start(p1, lo, hi, cfg, on_iteration=report("d1"))
    # components beyond the first half cost nothing there, so K itself stays
    # broad; the components inside the observed window must number two
    th1, off1 = first.theta.cpu().numpy(), first.offsets.cpu().numpy()
    seen = np.array([int(np.sum(th1[off1[i]:off1[i + 1], 1] < 0.45)) for i in range(N)])
    assert int(np.argmax(np.bincount(seen))) == 2, np.bincount(seen)
    p2 = lib.Problem(wl.PULSE, torch.tensor(d, device=dev), 0.0, dt, 1.0, k_hi, N, N * k_hi)
    cfg2 = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=150, seed=8, eps=lambda beta: 3e-4)
    post = smc.run_posterior_start(p2, split, first.offsets, first.theta, lo, hi, cfg2,
                                   on_iteration=report("post"))
    assert p2.get_bridge_split() == 0
    assert post.betas[-1] == 1.0
    k2 = np.array(post.k_hist[-1], dtype=float) / N
    assert int(np.argmax(k2)) == 3, k2
    prior = smc.run_prior_start(p2, lo, hi, smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=150,
                                                          seed=9), on_iteration=report("prior"))
    print(f"[smc] iterations: posterior-start {post.iterations}, prior-start {prior.iterations}",
          flush=True)
    assert post.iterations < prior.iterations


def test_metric_nuts_sharpens_the_component_posterior(lib, orc):
    """NUTS with the Gauss-Newton mass matrix (Sec. "No-U-Turn-Sampler") inside
    the same prior-start run: beta reaches one and the posterior over K puts
    more mass on the injected count than the identity-metric run, whose small
    raw-coordinate steps mix slowly (both runs share the seed and problem)."""
    T = 1000
    dt = 1.0 / (T - 1)
    inj = np.array([[5.0, 0.25, 0.02], [4.0, 0.52, 0.03], [5.5, 0.76, 0.015]])
    rng = np.random.default_rng(31)
    d = rng.standard_normal(T) + orc.template_sum(wl.PULSE, inj, T, 0.0, dt)
    N, k_hi = 2048, 6
    prob = lib.Problem(wl.PULSE, torch.tensor(d, device="cuda"), 0.0, dt, 1.0, k_hi, N, N * k_hi)
    lo = torch.tensor(wl.PULSE_PRIOR[:, 0].copy(), device="cuda")
    hi = torch.tensor(wl.PULSE_PRIOR[:, 1].copy(), device="cuda")
    print("[case] metric_smc", flush=True)
    out = {}
    for metric in (False, True):
        cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=150, seed=5, metric=metric)
        res = smc.run_prior_start(prob, lo, hi, cfg)
        final = np.array(res.k_hist[-1], dtype=float) / N
        print(f"[smc] metric={metric}: {res.iterations} iterations, K posterior {final.round(3)}, "
              f"log Z {res.log_evidence:.2f}", flush=True)
        assert res.betas[-1] == 1.0 and np.isfinite(res.log_evidence)
        th = res.theta.cpu().numpy()
        assert np.all(th >= wl.PULSE_PRIOR[:, 0]) and np.all(th <= wl.PULSE_PRIOR[:, 1])
        out[metric] = final
    assert int(np.argmax(out[True])) == 3 and out[True][3] >= 0.9, out[True]
    assert out[True][3] > out[False][3]


def test_posterior_start_with_the_metric(lib, orc):
    """The metric follows the bridge split, so the posterior-start mode can use
    it too: it ends at the full data's component count."""
    T, split = 1000, 500
    dt = 1.0 / (T - 1)
    inj = np.array([[5.0, 0.2, 0.02], [4.0, 0.36, 0.03], [5.5, 0.75, 0.015]])
    rng = np.random.default_rng(33)
    d = rng.standard_normal(T) + orc.template_sum(wl.PULSE, inj, T, 0.0, dt)
    N, k_hi = 2048, 6
    dev = "cuda"
    lo = torch.tensor(wl.PULSE_PRIOR[:, 0].copy(), device=dev)
    hi = torch.tensor(wl.PULSE_PRIOR[:, 1].copy(), device=dev)
    print("[case] posterior_start_metric", flush=True)
    p1 = lib.Problem(wl.PULSE, torch.tensor(d[:split], device=dev), 0.0, dt, 1.0, k_hi, N, N * k_hi)
    cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=150, seed=7, metric=True)
    first = smc.run_prior_start(p1, lo, hi, cfg)
    p2 = lib.Problem(wl.PULSE, torch.tensor(d, device=dev), 0.0, dt, 1.0, k_hi, N, N * k_hi)
    post = smc.run_posterior_start(p2, split, first.offsets, first.theta, lo, hi,
                                   smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=150, seed=8,
                                                 metric=True))
    k2 = np.array(post.k_hist[-1], dtype=float) / N
    print(f"[smc] posterior-start with metric: {post.iterations} iterations (first half "
          f"{first.iterations}), K posterior {k2.round(3)}", flush=True)
    assert post.betas[-1] == 1.0 and p2.get_bridge_split() == 0
    assert int(np.argmax(k2)) == 3 and k2[3] >= 0.8, k2


def test_gb_lisa_prior_start_recovers_the_number_of_binaries(lib, orc):
    """The frequency-domain Galactic-binary model (Sec. "LISA Galactic
    binaries": one year of noise-free A and E data) through the same driver
    with the per-source Gauss-Newton mass matrix: beta reaches one and the
    posterior over K peaks at the three injected binaries."""
    N, k_hi = 2048, 5
    w = wl.make_gblisa(N=N, k_lo=1, k_hi=k_hi, n_inj=3, noise=False, seed=503)
    d = orc.gblisa_spectrum(w.inj, w.T_obs, w.k0, w.B)
    dev = "cuda"
    prob = lib.Problem.frequency_domain(wl.GBLISA, torch.tensor(d, device=dev), w.k0, w.T_obs, w.S,
                                        k_hi, N, N * k_hi)
    lo = torch.tensor(wl.GBLISA_PRIOR[:, 0].copy(), device=dev)
    hi = torch.tensor(wl.GBLISA_PRIOR[:, 1].copy(), device=dev)
    print("[case] gb_lisa_smc", flush=True)
    cfg = smc.SMCConfig(N=N, k_lo=1, k_hi=k_hi, max_iters=300, seed=5, metric=True)
    res = smc.run_prior_start(prob, lo, hi, cfg)
    k = np.array(res.k_hist[-1], dtype=float) / N
    print(f"[smc] gb_lisa: {res.iterations} iterations, K posterior {k.round(3)}, "
          f"log Z {res.log_evidence:.1f}", flush=True)
    assert res.betas[-1] == 1.0 and np.isfinite(res.log_evidence)
    assert int(np.argmax(k)) == 3 and k[3] >= 0.9, k
    th = res.theta.cpu().numpy()
    assert np.all(th >= wl.GBLISA_PRIOR[:, 0]) and np.all(th <= wl.GBLISA_PRIOR[:, 1])


def test_gb_lisa_posterior_start_across_record_lengths(lib, orc):
    """The paper's Galactic-binary posterior-start (Sec. "LISA Galactic
    binaries"): a population sampled on six months of data is carried to
    twelve months by the bridge of eq. reuse_bridge between the two records.
    It must end at the injected count in fewer SMC iterations than a
    prior-start run on the twelve months."""
    N, k_hi = 2048, 5
    w = wl.make_gblisa(N=N, k_lo=1, k_hi=k_hi, n_inj=3, noise=False, seed=503)
    T2, T1 = w.T_obs, w.T_obs / 2
    k1 = wl.gblisa_band(T1)
    dev = "cuda"
    d1 = torch.tensor(orc.gblisa_spectrum(w.inj, T1, k1, w.B), device=dev)
    d2 = torch.tensor(orc.gblisa_spectrum(w.inj, T2, w.k0, w.B), device=dev)
    p1 = lib.Problem.frequency_domain(wl.GBLISA, d1, k1, T1, w.S, k_hi, N, N * k_hi)
    p2 = lib.Problem.frequency_domain(wl.GBLISA, d2, w.k0, T2, w.S, k_hi, N, N * k_hi)
    lo = torch.tensor(wl.GBLISA_PRIOR[:, 0].copy(), device=dev)
    hi = torch.tensor(wl.GBLISA_PRIOR[:, 1].copy(), device=dev)
    print("[case] gb_lisa_posterior_start", flush=True)
    cfg = dict(N=N, k_lo=1, k_hi=k_hi, max_iters=300, metric=True)
    first = smc.run_prior_start(p1, lo, hi, smc.SMCConfig(seed=11, **cfg))
    post = smc.run_bridge_start(p2, p1, first.offsets, first.theta, lo, hi,
                                smc.SMCConfig(seed=12, **cfg))
    prior = smc.run_prior_start(p2, lo, hi, smc.SMCConfig(seed=13, **cfg))
    k = np.array(post.k_hist[-1], dtype=float) / N
    print(f"[smc] gb_lisa: six months {first.iterations} iterations; twelve months "
          f"posterior-start {post.iterations}, prior-start {prior.iterations}; K posterior "
          f"{k.round(3)}", flush=True)
    assert post.betas[-1] == 1.0
    assert int(np.argmax(k)) == 3 and k[3] >= 0.8, k
    assert post.iterations < prior.iterations
