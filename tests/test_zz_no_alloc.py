"""logl_grad_batch_static (no handle, no allocation) against logl_grad_batch.

Two calls in a row share the device's static scratch; the second has a
smaller input, so it runs over what the first left behind. Each result is
compared with the handle-based entry point and with the FP64 oracle at the
parity tolerances.
"""
import sys

import numpy as np
import pytest
import torch

import parity as pm
from paper_2609_17674_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _case(lib, orc, w):
    d = pm.data_of(w)
    dd = pm.to_dev(d)
    off, th, be = pm.to_dev(w.offsets), pm.to_dev(w.theta.reshape(-1, w.P)), pm.to_dev(w.beta)
    ls, gs = lib.logl_grad_batch_static(w.model, dd, w.t_start, w.dt, w.sigma, w.k_max, off, th, be)
    torch.cuda.synchronize()
    prob = lib.Problem(w.model, dd, w.t_start, w.dt, w.sigma, w.k_max, w.N, max(w.M, 1))
    lh, gh = lib.logl_grad_batch(prob, off, th, be)
    torch.cuda.synchronize()
    prob.device_status()
    ref_l, ref_g = orc.logl_grad(w.model, d, w.t_start, w.dt, w.sigma, w.offsets, w.theta, w.beta)
    ls, gs, lh, gh = (x.cpu().numpy() for x in (ls, gs, lh, gh))
    pm.assert_logl(ls, lh, what="static vs handle logL")
    pm.assert_grad(w.model, w.offsets, w.theta, gs, gh, w.T, w.dt)
    pm.assert_logl(ls, ref_l, what="static vs oracle logL")
    pm.assert_grad(w.model, w.offsets, w.theta, gs, ref_g, w.T, w.dt)
    # the handle path's default tiling is the static one here: K > 0 particles agree bitwise
    K = np.diff(w.offsets)
    assert np.array_equal(ls[K > 0], lh[K > 0])
    assert np.array_equal(gs, gh)


@pytest.mark.parametrize("cfg,big,small", [
    ("pulse_batch", dict(N=600, T=5000), dict(N=70, T=1500)),
    ("gb_grad", dict(N=200, T=(1 << 13) + 777, k_hi=12), dict(N=40, T=3000, k_hi=6)),
])
def test_static_entry_point_matches_the_handle_path(lib, orc, cfg, big, small):
    for tag, ov in (("first", big), ("second, smaller", small)):
        w = wl.make_config(cfg, **ov)
        if w.model == wl.PULSE:
            w.beta = np.random.default_rng(9).random(w.N)
        say(cfg, tag, "N", w.N, "T", w.T, "M", w.M)
        _case(lib, orc, w)


def test_static_entry_point_with_longer_chunks_at_full_size(lib, orc):
    """The full sinusoid workload (T = 2^17, N = 4096, K up to 30): the handle
    path's default chunking would not fit the scratch, so the static form
    takes longer chunks; it agrees with the handle path on every particle and
    with the oracle on sampled ones, the largest K among them."""
    w = wl.make_config("gb_grad")
    say("gb_grad full size", "N", w.N, "T", w.T, "M", w.M)
    d = pm.data_of(w)
    dd = pm.to_dev(d)
    off, th, be = pm.to_dev(w.offsets), pm.to_dev(w.theta.reshape(-1, w.P)), pm.to_dev(w.beta)
    ls, gs = lib.logl_grad_batch_static(w.model, dd, w.t_start, w.dt, w.sigma, w.k_max, off, th, be)
    torch.cuda.synchronize()
    prob = lib.Problem(w.model, dd, w.t_start, w.dt, w.sigma, w.k_max, w.N, w.M)
    lh, gh = lib.logl_grad_batch(prob, off, th, be)
    torch.cuda.synchronize()
    prob.device_status()
    ls, gs, lh, gh = (x.cpu().numpy() for x in (ls, gs, lh, gh))
    pm.assert_logl(ls, lh, what="static vs handle logL")
    pm.assert_grad(w.model, w.offsets, w.theta, gs, gh, w.T, w.dt)
    K = np.diff(w.offsets)
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([rng.choice(w.N, 23, replace=False), [int(np.argmax(K))]]))
    sub = wl.subsample(w, idx)
    ref_l, ref_g = orc.logl_grad(w.model, d, w.t_start, w.dt, w.sigma, sub.offsets, sub.theta,
                                 sub.beta)
    rows = np.concatenate([np.arange(w.offsets[i], w.offsets[i + 1]) for i in idx])
    pm.assert_logl(ls[idx], ref_l, what="static vs oracle logL")
    pm.assert_grad(w.model, sub.offsets, sub.theta, gs[rows], ref_g, w.T, w.dt)


def test_static_entry_point_refuses_sizes_beyond_the_scratch(lib):
    say("static scratch limit")
    T = 1 << 24  # the FP32 copy of d alone exceeds the scratch
    d = torch.zeros(T, dtype=torch.float64, device="cuda")
    off = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    th = torch.tensor([[3.0, 0.5, 0.02]], dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SmcxError) as ei:
        lib.logl_grad_batch_static(wl.PULSE, d, 0.0, 1.0 / (T - 1), 1.0, 4, off, th)
    assert ei.value.code == lib.SMCX_ENOMEM and "static scratch" in str(ei.value)
