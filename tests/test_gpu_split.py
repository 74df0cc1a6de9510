"""The posterior-start bridge target (samples before the split untempered,
later ones tempered by beta) on the GPU against the oracle, through the C ABI."""
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


CASES = [
    # name, config, overrides, splits
    ("pulse", "pulse_batch", dict(N=200, T=4096, rj=True), (1000, 2048, 4095)),
    ("pulse_chunks", "pulse_batch", dict(N=80, T=9000, rj=True), (37, 4096, 6001)),
    ("gb", "gb_grad", dict(N=60, T=5000, k_hi=8, rj=True), (2500, 1)),
]


@pytest.mark.parametrize("name,cfg,ov,splits", CASES, ids=[c[0] for c in CASES])
def test_split_target_parity(lib, orc, name, cfg, ov, splits):
    w = wl.make_config(cfg, **ov)
    w.beta = np.random.default_rng(61).random(w.N)
    w.beta[::13] = 0.0
    d = pm.data_of(w)
    prob = lib.Problem(w.model, pm.to_dev(d), w.t_start, w.dt, w.sigma, w.k_max + 1, w.N, w.M)
    off, th, be = pm.to_dev(w.offsets), pm.to_dev(w.theta), pm.to_dev(w.beta)
    tb, di = w.extra["theta_birth"], w.extra["death_idx"]
    args = (w.model, d, w.t_start, w.dt, w.sigma, w.offsets, w.theta, w.beta)
    for split in splits:
        say(name, "split", split)
        prob.set_bridge_split(split)
        assert prob.get_bridge_split() == split
        rl, rg = orc.logl_grad_split(*args, split)
        rb, rd = orc.delta_split(*args, tb, di, split)
        for sorted_ in (1, 0):
            S = 16 if w.model == PULSE else 8
            chunk = 4096 if w.T > 4096 else 64 * S * ((w.T + 64 * S - 1) // (64 * S))
            prob.set_tiling(lib.KIND_GRAD, S, chunk, sorted_)
            prob.set_tiling(lib.KIND_LOGL, S, chunk, sorted_)
            prob.set_tiling(lib.KIND_DELTA, 8, chunk, sorted_)
            l, g = lib.logl_grad_batch(prob, off, th, be)
            l2 = lib.logl_batch(prob, off, th, be)
            db, dd = lib.delta_logl_birth_death(prob, off, th, be, pm.to_dev(tb), pm.to_dev(di))
            torch.cuda.synchronize()
            prob.device_status()
            l, g, l2, db, dd = (x.cpu().numpy() for x in (l, g, l2, db, dd))
            pm.assert_logl(l, rl)
            pm.assert_logl(l2, rl)
            pm.assert_grad(w.model, w.offsets, w.theta, g, rg, w.T, w.dt)
            # birth/death: the condition scale of the untempered-plus-tempered sums
            sb = pm.delta_scale(w.model, w, list(tb), np.ones(w.N), w.sigma, rb)
            rows = [w.theta[w.offsets[i] + di[i]] if di[i] >= 0 else None for i in range(w.N)]
            sd = pm.delta_scale(w.model, w, rows, np.ones(w.N), w.sigma, rd)
            assert np.all(np.abs(db - rb) <= 1e-6 * sb)
            assert np.all(np.abs(dd - rd) <= 1e-6 * sd)
    # split 0 is the prior bridge, bit for bit the same as without ever setting one
    prob.set_bridge_split(0)
    l0, g0 = lib.logl_grad_batch(prob, off, th, be)
    fresh = lib.Problem(w.model, pm.to_dev(d), w.t_start, w.dt, w.sigma, w.k_max + 1, w.N, w.M)
    for kind in (lib.KIND_GRAD, lib.KIND_LOGL, lib.KIND_DELTA):
        fresh.set_tiling(kind, *prob.get_tiling(kind))
    l1, g1 = lib.logl_grad_batch(fresh, off, th, be)
    torch.cuda.synchronize()
    assert torch.equal(l0, l1) and torch.equal(g0, g1)


def test_split_leapfrog_and_nuts_graph_follow_the_split(lib, orc):
    w = wl.make_config("pulse_mutate", N=120, T=2048, seed=62)
    d = pm.data_of(w)
    prob = lib.Problem(w.model, pm.to_dev(d), w.t_start, w.dt, w.sigma, w.k_max, w.N, w.M)
    off, th, be = pm.to_dev(w.offsets), pm.to_dev(w.theta), pm.to_dev(w.beta)
    rng = np.random.default_rng(63)
    p0 = rng.standard_normal(w.theta.shape)
    eps = 1e-4
    for split in (700, 1500):
        say("split leapfrog", split)
        prob.set_bridge_split(split)
        l0, g0 = lib.logl_grad_batch(prob, off, th, be)
        q1, p1, g1, l1 = lib.leapfrog(prob, off, be, eps, th, pm.to_dev(p0), g0)
        torch.cuda.synchronize()
        q1, p1, g1, l1 = (x.cpu().numpy() for x in (q1, p1, g1, l1))
        rq, rp, rl, rg = orc.leapfrog_split(w.model, d, w.t_start, w.dt, w.sigma, w.offsets,
                                            w.theta, p0, w.beta, eps, split)
        _, rg0 = orc.logl_grad_split(w.model, d, w.t_start, w.dt, w.sigma, w.offsets, w.theta,
                                     w.beta, split)
        pm.assert_logl(l1, rl)
        pm.assert_grad(w.model, w.offsets, rq, g1, rg, w.T, w.dt)
        # the drift carries the start gradient's tolerance: eps^2/2 times its error
        tol_q = 0.5 * eps * eps * 1e-4 * np.abs(rg0).max() + 1e-14 * np.abs(rq)
        assert np.all(np.abs(q1 - rq) <= tol_q)
    # a NUTS graph captured at one split must not be replayed at another
    D = 4
    lib.nuts_reserve(prob, D)
    mom, dirs, ul, ut = (pm.to_dev(x) for x in wl.nuts_draws(w.N, w.M, w.P, D, 64))
    lo = pm.to_dev(wl.PULSE_PRIOR[:, 0].copy())
    hi = pm.to_dev(wl.PULSE_PRIOR[:, 1].copy())
    res = {}
    for split, graph in ((700, True), (1500, True), (1500, False)):
        say("split nuts", split, graph)
        prob.set_bridge_split(split)
        l0, g0 = lib.logl_grad_batch(prob, off, th, be)
        q, l, g = th.clone(), l0.clone(), g0.clone()
        lib.nuts_transition(prob, off, be, 2e-4, D, q, l, g, mom, dirs, ul, ut, lo, hi,
                            use_graph=graph)
        torch.cuda.synchronize()
        res[(split, graph)] = [x.cpu().numpy() for x in (q, l, g)]
    for x, y in zip(res[(1500, True)], res[(1500, False)]):
        assert np.array_equal(x, y)
    assert not np.array_equal(res[(700, True)][1], res[(1500, True)][1])


def test_split_leaves_reweighting_and_rejects_the_plain_form(lib, orc):
    w = wl.make_config("gb_grad", N=30, T=3000, k_hi=6, seed=65)
    d = pm.data_of(w)
    prob = lib.Problem(w.model, pm.to_dev(d), w.t_start, w.dt, w.sigma, w.k_max, w.N, w.M)
    off, th = pm.to_dev(w.offsets), pm.to_dev(w.theta)
    a = lib.reweight_extend(prob, 1000, 3000, off, th, 0.4)
    prob.set_bridge_split(1200)
    b = lib.reweight_extend(prob, 1000, 3000, off, th, 0.4)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    with pytest.raises(lib.SmcxError, match="prior bridge"):
        lib.plain_logl_grad(prob, w.offsets, th)
    with pytest.raises(lib.SmcxError):
        prob.set_bridge_split(w.T + 1)
