"""The LISA Galactic-binary model (frequency domain) on the GPU against the
oracle, through the C ABI.

Tolerance, from the arithmetic: both sides evaluate the same definitions in
FP64 (the GPU with a radix-2 FFT, the oracle with a direct 64-point sum and
libm), so templates agree to a few hundred ulp of the largest bin. The
residual in a bin is at least about the noise there, at most about 20 times
smaller than the template, so logL agrees to well under 1e-10 relative and
the gradient (natural coordinates: f0 T_obs, fdot T_obs^2, the rest as they
are) to 1e-8 of its norm. The bounds used are 1e-9 and 1e-7.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2609_17674_amd import workloads as wl

pytestmark = pytest.mark.gpu
GBLISA = wl.GBLISA
NAT = np.array([wl.GBLISA_T_OBS, wl.GBLISA_T_OBS ** 2, 1, 1, 1, 1, 1, 1], dtype=float)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x), device="cuda")
    return t if dtype is None else t.to(dtype)


def _data(orc, w):
    return w.noise + orc.gblisa_spectrum(w.inj, w.T_obs, w.k0, w.B)


def _problem(lib, w, d):
    return lib.Problem.frequency_domain(GBLISA, dev(d), w.k0, w.T_obs, w.S, w.k_max, w.N,
                                        max(w.M, 1))


def test_template_spectrum_matches_oracle(lib, orc):
    say("gblisa_spectrum")
    w = wl.make_gblisa(N=4, n_inj=10, seed=400)
    # include sources whose windows leave the band on either side
    th = np.vstack([w.inj, w.inj[:2]])
    th[-2, 0] = (w.k0 + 5) / w.T_obs
    th[-1, 0] = (w.k0 + w.B - 3) / w.T_obs
    for B in (w.B, 77, 200):
        got = lib.template_spectrum(GBLISA, dev(th), w.T_obs, w.k0, B).cpu().numpy()
        ref = orc.gblisa_spectrum(th, w.T_obs, w.k0, B)
        assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref)), B


@pytest.mark.parametrize("noise,beta", [(True, "uniform"), (False, "one")], ids=["noise", "noisefree"])
def test_logl_and_gradient_match_oracle(lib, orc, noise, beta):
    w = wl.make_gblisa(N=300, k_lo=0, k_hi=10, n_inj=6, beta=beta, noise=noise, seed=401)
    say("gblisa_logl_grad", noise, beta, "N", w.N, "M", w.M)
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    l_only = lib.logl_batch(prob, off, th, be)
    l, g = lib.logl_grad_batch(prob, off, th, be)
    torch.cuda.synchronize()
    prob.device_status()
    l_only, l, g = l_only.cpu().numpy(), l.cpu().numpy(), g.cpu().numpy()
    rl, rg = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, w.offsets, w.theta, w.beta)
    assert np.array_equal(l, l_only)
    assert np.all(np.abs(l - rl) <= 1e-9 * np.abs(rl) + 1e-300)
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        if a == b:
            continue
        gn, rn = (g[a:b] / NAT).reshape(-1), (rg[a:b] / NAT).reshape(-1)
        assert np.linalg.norm(gn - rn) <= 1e-7 * np.linalg.norm(rn) + 1e-300, i


def test_birth_death_match_oracle(lib, orc):
    w = wl.make_gblisa(N=200, k_lo=0, k_hi=8, n_inj=5, beta="uniform", noise=True, seed=402)
    say("gblisa_delta")
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    tb, di = w.extra["theta_birth"], w.extra["death_idx"]
    db, dd = lib.delta_logl_birth_death(prob, dev(w.offsets), dev(w.theta), dev(w.beta), dev(tb),
                                        dev(di))
    torch.cuda.synchronize()
    prob.device_status()
    rb, rd = orc.gblisa_delta(d, w.k0, w.T_obs, w.S, w.offsets, w.theta, w.beta, tb, di)
    db, dd = db.cpu().numpy(), dd.cpu().numpy()
    # condition-scaled: 1e-9 of |<r, h>| + |h|^2 / 2, which bounds both terms
    l0 = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, w.offsets, w.theta, w.beta, grad=False)
    scale = np.abs(rb) + np.abs(rd) + 1e-6 * np.abs(l0) + 1.0
    assert np.all(np.abs(db - rb) <= 1e-9 * scale)
    assert np.all(np.abs(dd - rd) <= 1e-9 * scale)
    assert np.all(dd[di == -1] == 0.0)


# carrier bins relative to the band's first bin: windows that overlap either
# edge, lie just outside it, or are far from it (beyond the kernels' clamp of
# the window start to [-128, B])
EDGE_OFFSETS = (-100000, -500, -97, -64, -63, -33, -31, 0, 31, 97, 98, 127, 128, 160, 161, 300,
                1000000)


def test_sources_outside_the_band(lib, orc):
    w = wl.make_gblisa(N=96, k_lo=1, k_hi=6, n_inj=6, beta="uniform", noise=True, seed=420)
    say("gblisa_edges", "N", w.N, "M", w.M)
    th, tb = w.theta.copy(), w.extra["theta_birth"].copy()
    # the first source of each particle and each particle's birth candidate
    # take the edge bins in turn (f0 inside its bin)
    for i in range(w.N):
        off = EDGE_OFFSETS[i % len(EDGE_OFFSETS)]
        th[w.offsets[i], 0] = (w.k0 + off + 0.37) / w.T_obs
        tb[i, 0] = (w.k0 + EDGE_OFFSETS[(i + 5) % len(EDGE_OFFSETS)] + 0.61) / w.T_obs
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    off, be = dev(w.offsets), dev(w.beta)
    l, g = lib.logl_grad_batch(prob, off, dev(th), be)
    db, dd = lib.delta_logl_birth_death(prob, off, dev(th), be, dev(tb), dev(w.extra["death_idx"]))
    torch.cuda.synchronize()
    prob.device_status()
    l, g, db, dd = (x.cpu().numpy() for x in (l, g, db, dd))
    rl, rg = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, w.offsets, th, w.beta)
    rb, rd = orc.gblisa_delta(d, w.k0, w.T_obs, w.S, w.offsets, th, w.beta, tb, w.extra["death_idx"])
    assert np.all(np.isfinite(l)) and np.all(np.isfinite(g))
    assert np.all(np.abs(l - rl) <= 1e-9 * np.abs(rl))
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        gn, rn = (g[a:b] / NAT).reshape(-1), (rg[a:b] / NAT).reshape(-1)
        assert np.linalg.norm(gn - rn) <= 1e-7 * np.linalg.norm(rn), i
        # a window wholly outside the band has no gradient
        q = int(np.floor(th[a, 0] * w.T_obs)) - w.k0
        if q + 32 <= 0 or q - 32 >= w.B:
            assert np.all(g[a] == 0.0) and np.all(rg[a] == 0.0), i
    scale = np.abs(rb) + np.abs(rd) + 1e-6 * np.abs(rl) + 1.0
    assert np.all(np.abs(db - rb) <= 1e-9 * scale)
    assert np.all(np.abs(dd - rd) <= 1e-9 * scale)


@pytest.mark.parametrize("B", [1, 7, 40, 64, 65])
def test_bands_narrower_than_a_window(lib, orc, B):
    """Bands of fewer bins than a source's 64-bin window (and one just
    wider): every window is cut by the band on one or both sides."""
    w = wl.make_gblisa(N=64, k_lo=0, k_hi=6, n_inj=4, beta="uniform", noise=False, seed=440 + B)
    # a band of B bins around the carrier bin of one injection, with the
    # injections and white noise of those bins
    k0 = int(np.floor(w.inj[1, 0] * w.T_obs)) - B // 2
    d = orc.gblisa_spectrum(w.inj, w.T_obs, k0, B)
    rng = np.random.default_rng(450 + B)
    sd = np.sqrt(w.S * w.T_obs / 4.0)
    d = d + sd * (rng.standard_normal(d.shape) + 1j * rng.standard_normal(d.shape))
    say("gblisa_narrow_band", "B", B, "k0", k0, "N", w.N, "M", w.M)
    prob = lib.Problem.frequency_domain(GBLISA, dev(d), k0, w.T_obs, w.S, w.k_max, w.N, max(w.M, 1))
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    l, g = lib.logl_grad_batch(prob, off, th, be)
    tb, di = w.extra["theta_birth"], w.extra["death_idx"]
    db, dd = lib.delta_logl_birth_death(prob, off, th, be, dev(tb), dev(di))
    torch.cuda.synchronize()
    prob.device_status()
    l, g, db, dd = (x.cpu().numpy() for x in (l, g, db, dd))
    rl, rg = orc.gblisa_logl_grad(d, k0, w.T_obs, w.S, w.offsets, w.theta, w.beta)
    rb, rd = orc.gblisa_delta(d, k0, w.T_obs, w.S, w.offsets, w.theta, w.beta, tb, di)
    # the band meets the windows of most sources
    assert np.count_nonzero(rg[:, 0]) > w.M // 2
    assert np.all(np.abs(l - rl) <= 1e-9 * np.abs(rl) + 1e-300)
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        if a == b:
            continue
        gn, rn = (g[a:b] / NAT).reshape(-1), (rg[a:b] / NAT).reshape(-1)
        assert np.linalg.norm(gn - rn) <= 1e-7 * np.linalg.norm(rn) + 1e-300, i
    scale = np.abs(rb) + np.abs(rd) + 1e-6 * np.abs(rl) + 1.0
    assert np.all(np.abs(db - rb) <= 1e-9 * scale)
    assert np.all(np.abs(dd - rd) <= 1e-9 * scale)


def test_particles_with_many_sources(lib, orc):
    """K up to 40: many sources per particle through the forward pass, the
    adjoint, birth/death and the metric (one lane per source in the pass that
    prepares their constants)."""
    w = wl.make_gblisa(N=40, k_lo=14, k_hi=40, n_inj=6, beta="uniform", noise=True, seed=430)
    say("gblisa_many_sources", "N", w.N, "M", w.M, "K max", int(w.K.max()))
    assert w.K.max() > 32 and w.K.min() <= 16
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    l, g = lib.logl_grad_batch(prob, off, th, be)
    tb, di = w.extra["theta_birth"], w.extra["death_idx"]
    db, dd = lib.delta_logl_birth_death(prob, off, th, be, dev(tb), dev(di))
    fo, F = lib.gauss_newton_metric(prob, off, th, be)
    torch.cuda.synchronize()
    prob.device_status()
    l, g, db, dd = l.cpu().numpy(), g.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy()
    fo, F = fo.cpu().numpy(), F.cpu().numpy()
    rl, rg = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, w.offsets, w.theta, w.beta)
    assert np.all(np.abs(l - rl) <= 1e-9 * np.abs(rl))
    rb, rd = orc.gblisa_delta(d, w.k0, w.T_obs, w.S, w.offsets, w.theta, w.beta, tb, di)
    scale = np.abs(rb) + np.abs(rd) + 1e-6 * np.abs(rl) + 1.0
    assert np.all(np.abs(db - rb) <= 1e-9 * scale)
    assert np.all(np.abs(dd - rd) <= 1e-9 * scale)
    ref = orc.gblisa_fisher(w.k0, w.B, w.T_obs, w.S, w.offsets, w.theta, w.beta)
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        gn, rn = (g[a:b] / NAT).reshape(-1), (rg[a:b] / NAT).reshape(-1)
        assert np.linalg.norm(gn - rn) <= 1e-7 * np.linalg.norm(rn), i
        n = 8 * (b - a)
        got = F[fo[i]:fo[i + 1]].reshape(n, n)
        dg = np.sqrt(np.diag(ref[i]))
        assert np.all(np.abs(got - ref[i]) <= 1e-9 * np.outer(dg, dg)), i


@pytest.mark.parametrize("B,k_hi", [(128, 10), (200, 40)], ids=["band128", "band200_K40"])
def test_few_listed_particles_share_a_workgroup(lib, orc, B, k_hi):
    """A gradient launch over few listed particles gives each particle a whole
    workgroup, whose waves take every fourth source: logL, gradient and the
    leapfrog step equal, bit for bit, those of the same particles as a
    population of their own (one wave per particle), and match the oracle."""
    base = wl.make_gblisa(N=24, k_lo=1, k_hi=k_hi, n_inj=6, beta="uniform", noise=False,
                          seed=431)
    d = orc.gblisa_spectrum(base.inj, base.T_obs, base.k0, B)
    n_big = 600
    idx = np.sort(np.random.default_rng(432).choice(n_big, size=base.N, replace=False))
    counts = np.zeros(n_big, dtype=np.int64)
    counts[idx] = base.K
    off_big = np.concatenate([[0], np.cumsum(counts)])
    beta_big = np.full(n_big, 0.5)
    beta_big[idx] = base.beta
    say("gblisa_split", "B", B, "K max", int(base.K.max()), "listed", base.N, "of", n_big)
    rng = np.random.default_rng(433)
    scales = np.array([0.05 / base.T_obs, 1e-19, 0.02, 0.02, 0.02, 0.02, 0.02, 0.05])
    eps = 1e-17
    p0 = 0.5 * rng.standard_normal(base.theta.shape) * scales / eps
    dirs = np.where(rng.random(base.N) < 0.5, -1, 1).astype(np.int8)
    dirs_big = np.ones(n_big, dtype=np.int8)
    dirs_big[idx] = dirs
    out = []
    for N, off, be, di in ((base.N, base.offsets, base.beta, dirs),
                           (n_big, off_big, beta_big, dirs_big)):
        prob = lib.Problem.frequency_domain(GBLISA, dev(d), base.k0, base.T_obs, base.S,
                                            base.k_max, N, base.M)
        o, th, b = dev(off), dev(base.theta), dev(be)
        l, g = lib.logl_grad_batch(prob, o, th, b)
        q1, p1, g1, l1 = lib.leapfrog(prob, o, b, eps, th, dev(p0), g, dir=dev(di))
        torch.cuda.synchronize()
        prob.device_status()
        out.append([x.cpu().numpy() for x in (l, g, q1, p1, g1, l1)])
    (l, g, q1, p1, g1, l1), (lb, gb, q1b, p1b, g1b, l1b) = out
    assert np.array_equal(lb[idx], l) and np.array_equal(l1b[idx], l1)
    for x, y in ((g, gb), (q1, q1b), (p1, p1b), (g1, g1b)):
        assert np.array_equal(x, y)
    rl, rg = orc.gblisa_logl_grad(d, base.k0, base.T_obs, base.S, base.offsets, base.theta,
                                  base.beta)
    assert np.all(np.abs(l - rl) <= 1e-9 * np.abs(rl))
    for i in range(base.N):
        a, b = base.offsets[i], base.offsets[i + 1]
        gn, rn = (g[a:b] / NAT).reshape(-1), (rg[a:b] / NAT).reshape(-1)
        assert np.linalg.norm(gn - rn) <= 1e-7 * np.linalg.norm(rn), i


def _nuts_gb(lib, d, w, N, off, theta, beta, D, eps, draws, W):
    """One GB NUTS transition (block mass matrix W [M, 8, 8]); numpy results."""
    mom, dirs, ul, ut = draws
    prob = lib.Problem.frequency_domain(GBLISA, dev(d), w.k0, w.T_obs, w.S, w.k_max, N,
                                        theta.shape[0])
    lib.nuts_reserve(prob, D)
    o, th, be = dev(off), dev(theta), dev(beta)
    l, g = lib.logl_grad_batch(prob, o, th, be)
    q = th.clone()
    depth, steps, status = lib.nuts_transition(prob, o, be, eps, D, q, l, g, dev(mom), dev(dirs),
                                               dev(ul), dev(ut), metric_blocks=dev(W))
    torch.cuda.synchronize()
    prob.device_status()
    return [x.cpu().numpy() for x in (q, l, g, depth, steps, status)]


def test_nuts_late_doublings_step_through_the_listed_particles(lib, orc):
    """From the third doubling on, the NUTS gradient, leaf and merge launches
    take fixed grids whose workgroups step through the listed particles, and
    few listed particles share workgroups. Per-particle results do not
    depend on that: a population of 12000 (more particles still extending
    than one pass of the grid holds) equals, bit for bit, its two halves
    run alone (one pass each); 24 particles among 576 with K = 0 (a
    workgroup each) equal the 24 alone."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    D, eps = 3, 0.05
    scales = np.array([0.05 / wl.GBLISA_T_OBS, 1e-19, 0.02, 0.02, 0.02, 0.02, 0.02, 0.05])
    w = wl.make_gblisa(N=12000, k_lo=1, k_hi=3, n_inj=6, beta="uniform", noise=True, seed=434)
    d = _data(orc, w)
    draws = wl.nuts_draws(w.N, w.M, 8, D, seed=435)
    W = np.broadcast_to(np.diag(scales), (w.M, 8, 8)).copy()
    say("gblisa_nuts_strided", "N", w.N, "M", w.M, "CUs", n_cu)
    full = _nuts_gb(lib, d, w, w.N, w.offsets, w.theta, w.beta, D, eps, draws, W)
    assert np.sum(full[3] >= D) > 6 * n_cu * 4  # more than one pass at the last doubling
    h = w.N // 2
    parts = []
    for lo, hi in ((0, h), (h, w.N)):
        a, b = w.offsets[lo], w.offsets[hi]
        sub = (draws[0][a:b], draws[1][lo:hi], draws[2][lo:hi], draws[3][lo:hi])
        parts.append(_nuts_gb(lib, d, w, hi - lo, w.offsets[lo:hi + 1] - a, w.theta[a:b],
                              w.beta[lo:hi], D, eps, sub, W[a:b]))
    for x, y0, y1 in zip(full, *parts):
        assert np.array_equal(x, np.concatenate([y0, y1]))
    # few listed particles among many without sources
    m = 24
    few = wl.make_gblisa(N=m, k_lo=1, k_hi=3, n_inj=6, beta="uniform", noise=True, seed=436)
    fd_ = _data(orc, few)
    fdraws = wl.nuts_draws(m, few.M, 8, D, seed=437)
    fW = np.broadcast_to(np.diag(scales), (few.M, 8, 8)).copy()
    alone = _nuts_gb(lib, fd_, few, m, few.offsets, few.theta, few.beta, D, eps, fdraws, fW)
    n_big = 600
    idx = np.sort(np.random.default_rng(438).choice(n_big, size=m, replace=False))
    counts = np.zeros(n_big, dtype=np.int64)
    counts[idx] = few.K
    off_big = np.concatenate([[0], np.cumsum(counts)])
    beta_big = np.full(n_big, 0.5)
    beta_big[idx] = few.beta
    dirs_big = np.ones((n_big, D), dtype=np.int8)
    dirs_big[idx] = fdraws[1]
    ul_big = np.full((n_big, (1 << D) - 1), 0.5)
    ul_big[idx] = fdraws[2]
    ut_big = np.full((n_big, D), 0.5)
    ut_big[idx] = fdraws[3]
    among = _nuts_gb(lib, fd_, few, n_big, off_big, few.theta, beta_big, D, eps,
                     (fdraws[0], dirs_big, ul_big, ut_big), fW)
    assert np.array_equal(among[0], alone[0]) and np.array_equal(among[2], alone[2])
    for k in (1, 3, 4, 5):
        assert np.array_equal(among[k][idx], alone[k])


def test_invalid_particles_and_refusals(lib, orc):
    w = wl.make_gblisa(N=6, k_lo=1, k_hi=3, n_inj=2, seed=403)
    say("gblisa_invalid")
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    off = w.offsets.copy()
    off[3] = off[2] - 1  # non-monotone
    l = lib.logl_batch(prob, dev(off), dev(w.theta), dev(w.beta))
    torch.cuda.synchronize()
    with pytest.raises(lib.SmcxError):
        prob.device_status()
    assert np.isnan(l.cpu().numpy()[2])
    with pytest.raises(lib.SmcxError, match="time-domain"):
        lib.reweight_extend(prob, 0, 1, dev(w.offsets), dev(w.theta), 0.1)
    with pytest.raises(lib.SmcxError, match="tiling"):
        prob.set_tiling(lib.KIND_GRAD, 16, 1024, 1)
    with pytest.raises(lib.SmcxError, match="split"):
        prob.set_bridge_split(1)


def test_nuts_depth_one_on_the_frequency_domain_model(lib, orc):
    """One NUTS leaf on the GB model: a leapfrog step with the oracle's
    gradients, with a diagonal mass matrix (W = diag of per-parameter
    scales), then the acceptance on exp(H0 - H1)."""
    w = wl.make_gblisa(N=64, k_lo=1, k_hi=4, n_inj=4, beta="half", noise=True, seed=404)
    say("gblisa_nuts_depth1")
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    lib.nuts_reserve(prob, 1)
    scales = np.array([0.05 / w.T_obs, 1e-19, 0.02, 0.02, 0.02, 0.02, 0.02, 0.05])
    Wb = [np.diag(np.tile(scales, int(k))) for k in w.K]
    wo, Wp = wl.pack_blocks(Wb)
    mom, dirs, ul, ut = wl.nuts_draws(w.N, w.M, 8, 1, seed=405)
    ul[:] = 0.0
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    l0, g0 = lib.logl_grad_batch(prob, off, th, be)
    q, l, g = th.clone(), l0.clone(), g0.clone()
    eps = 0.4
    _, steps, status = lib.nuts_transition(prob, off, be, eps, 1, q, l, g, dev(mom), dev(dirs),
                                           dev(ul), dev(ut), metric=(dev(wo), dev(Wp)))
    torch.cuda.synchronize()
    prob.device_status()
    q, status = q.cpu().numpy(), status.cpu().numpy()
    rl0, rg0 = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, w.offsets, w.theta, w.beta)
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        Wi = Wb[i]
        e = eps * dirs[i, 0]
        r0 = mom[a:b].reshape(-1)
        rh = r0 + 0.5 * e * Wi @ rg0[a:b].reshape(-1)
        q1 = w.theta[a:b].reshape(-1) + e * Wi.T @ rh
        l1, g1 = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, [0, b - a], q1.reshape(-1, 8),
                                      w.beta[i:i + 1])
        r1 = rh + 0.5 * e * Wi @ g1.reshape(-1)
        H0 = -rl0[i] + 0.5 * r0 @ r0
        H1 = -l1[0] + 0.5 * r1 @ r1
        if not H1 - H0 <= 1000:
            assert status[i] == 2
            continue
        accept = ut[i, 0] < np.exp(min(H0 - H1, 0.0))  # min(1, e^(H0-H1)) without overflow
        ref = q1 if accept else w.theta[a:b].reshape(-1)
        # the kicks differ by the gradient bound (1e-7 of the natural norm),
        # far below 1e-6 of a step's scale
        tol = 1e-12 * np.abs(ref) + 1e-6 * np.tile(scales, b - a)
        assert np.all(np.abs(q[a:b].reshape(-1) - ref) <= tol), i


def test_metric_matches_oracle(lib, orc):
    """Per-source Gauss-Newton blocks (both sides FP64; the GPU sums the
    envelope derivatives over the 64 samples, the oracle the derivative
    spectra over the band, equal by Parseval while windows lie inside it)."""
    w = wl.make_gblisa(N=120, k_lo=0, k_hi=6, n_inj=4, beta="uniform", noise=True, seed=406)
    say("gblisa_metric")
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    fo, F = lib.gauss_newton_metric(prob, dev(w.offsets), dev(w.theta), dev(w.beta))
    torch.cuda.synchronize()
    prob.device_status()
    fo, F = fo.cpu().numpy(), F.cpu().numpy()
    ref = orc.gblisa_fisher(w.k0, w.B, w.T_obs, w.S, w.offsets, w.theta, w.beta)
    for i in range(w.N):
        n = 8 * int(w.K[i])
        if n == 0:
            continue
        got = F[fo[i]:fo[i + 1]].reshape(n, n)
        dg = np.sqrt(np.diag(ref[i]))
        assert np.all(np.abs(got - ref[i]) <= 1e-9 * np.outer(dg, dg)), i
        mask = np.kron(np.eye(n // 8), np.ones((8, 8))) == 0
        assert np.all(got[mask] == 0.0)


def test_factor_with_eight_parameters(lib, orc):
    """Blocks of the eight-parameter model that are singular in the last
    three parameters of every source (as the metric of a face-on source is)
    and definite only through the ridge on those parameters."""
    say("gblisa_factor")
    K = np.array([3, 0, 1, 5, 2])
    off = np.concatenate([[0], np.cumsum(K)])
    blocks = wl.spd_blocks(K * 8, seed=410, spread=3.0)
    for b, k in zip(blocks, K):
        for j in range(int(k)):
            sl = slice(8 * j + 5, 8 * j + 8)
            b[sl, :] = 0.0
            b[:, sl] = 0.0
    ridge = np.array([1e-3, 1e-2, 0.5, 0.7, 0.3, 1.2, 1.2, 0.3])
    fo, Fp = wl.pack_blocks(blocks)
    w = wl.make_gblisa(N=len(K), k_hi=int(K.max()), n_inj=1, seed=411)
    prob = lib.Problem.frequency_domain(GBLISA, dev(w.noise), w.k0, w.T_obs, w.S, int(K.max()),
                                        len(K), int(off[-1]))
    W = lib.metric_factor(prob, dev(off), dev(fo), dev(Fp), ridge)
    torch.cuda.synchronize()
    prob.device_status()
    Wg = W.cpu().numpy()
    ref, status = orc.metric_factor(GBLISA, off, blocks, ridge)
    assert np.all(status == 0)
    for i, (blk, r) in enumerate(zip(blocks, ref)):
        n = blk.shape[0]
        if n == 0:
            continue
        g = Wg[fo[i]:fo[i + 1]].reshape(n, n)
        D = np.sqrt(np.diag(blk) + np.tile(ridge, K[i]))
        gd, rd = g * D, r * D
        assert np.all(np.abs(gd - rd) <= 1e-10 * np.abs(rd).max(axis=1, keepdims=True)), i


def test_full_size_population_on_sampled_particles(lib, orc):
    """The benchmark's configuration (N = 40000, K ~ U{1..10}, ten noise-free
    binaries, one year) in one launch; particles sampled for the oracle."""
    w = wl.make_gblisa(N=40000, k_lo=1, k_hi=10, n_inj=10, beta="uniform", noise=False)
    say("gblisa_full_size", "M", w.M)
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    l, g = lib.logl_grad_batch(prob, dev(w.offsets), dev(w.theta), dev(w.beta))
    torch.cuda.synchronize()
    prob.device_status()
    l, g = l.cpu().numpy(), g.cpu().numpy()
    rng = np.random.default_rng(407)
    idx = np.sort(rng.choice(w.N, size=400, replace=False))
    for i in idx:
        a, b = w.offsets[i], w.offsets[i + 1]
        rl, rg = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, [0, b - a], w.theta[a:b],
                                      w.beta[i:i + 1])
        assert abs(l[i] - rl[0]) <= 1e-9 * abs(rl[0]), i
        gn, rn = (g[a:b] / NAT).reshape(-1), (rg / NAT).reshape(-1)
        assert np.linalg.norm(gn - rn) <= 1e-7 * np.linalg.norm(rn), i


def test_bridge_between_two_records(lib, orc):
    """Eq. reuse_bridge between a six-month and a twelve-month record: every
    tempered call evaluates (1 - beta) logL_6 + beta logL_12 (gradient,
    birth/death and metric alike); clearing the partner restores the
    twelve-month handle bit for bit."""
    w = wl.make_gblisa(N=150, k_lo=0, k_hi=6, n_inj=4, beta="uniform", noise=False, seed=420)
    say("gblisa_bridge")
    T2, T1 = w.T_obs, w.T_obs / 2
    k1 = wl.gblisa_band(T1)
    d2 = orc.gblisa_spectrum(w.inj, T2, w.k0, w.B)
    d1 = orc.gblisa_spectrum(w.inj, T1, k1, w.B)
    p2 = _problem(lib, w, d2)
    p1 = lib.Problem.frequency_domain(GBLISA, dev(d1), k1, T1, w.S, w.k_max, w.N, max(w.M, 1))
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    plain_l, plain_g = lib.logl_grad_batch(p2, off, th, be)
    p2.set_bridge_partner(p1)
    l, g = lib.logl_grad_batch(p2, off, th, be)
    tb, di = w.extra["theta_birth"], w.extra["death_idx"]
    db, dd = lib.delta_logl_birth_death(p2, off, th, be, dev(tb), dev(di))
    fo, F = lib.gauss_newton_metric(p2, off, th, be)
    torch.cuda.synchronize()
    p2.device_status()
    l, g, db, dd = (x.cpu().numpy() for x in (l, g, db, dd))
    fo, F = fo.cpu().numpy(), F.cpu().numpy()
    b = w.beta
    r1l, r1g = orc.gblisa_logl_grad(d1, k1, T1, w.S, w.offsets, w.theta, np.ones(w.N))
    r2l, r2g = orc.gblisa_logl_grad(d2, w.k0, T2, w.S, w.offsets, w.theta, np.ones(w.N))
    rl = (1 - b) * r1l + b * r2l
    assert np.all(np.abs(l - rl) <= 1e-9 * (np.abs(r1l) + np.abs(r2l)))
    rows = np.repeat(np.arange(w.N), w.K)
    rg = (1 - b[rows])[:, None] * r1g + b[rows][:, None] * r2g
    for i in range(w.N):
        a, c = w.offsets[i], w.offsets[i + 1]
        if a == c:
            continue
        scale = np.linalg.norm((np.abs(r1g[a:c]) + np.abs(r2g[a:c])) / NAT)
        assert np.linalg.norm((g[a:c] - rg[a:c]) / NAT) <= 1e-7 * scale, i
    b1, dd1 = orc.gblisa_delta(d1, k1, T1, w.S, w.offsets, w.theta, np.ones(w.N), tb, di)
    b2, dd2 = orc.gblisa_delta(d2, w.k0, T2, w.S, w.offsets, w.theta, np.ones(w.N), tb, di)
    sc = np.abs(b1) + np.abs(b2) + np.abs(dd1) + np.abs(dd2) + 1.0
    assert np.all(np.abs(db - ((1 - b) * b1 + b * b2)) <= 1e-9 * sc)
    assert np.all(np.abs(dd - ((1 - b) * dd1 + b * dd2)) <= 1e-9 * sc)
    F1 = orc.gblisa_fisher(k1, w.B, T1, w.S, w.offsets, w.theta, np.ones(w.N))
    F2 = orc.gblisa_fisher(w.k0, w.B, T2, w.S, w.offsets, w.theta, np.ones(w.N))
    for i in range(w.N):
        n = 8 * int(w.K[i])
        if n == 0:
            continue
        ref = (1 - b[i]) * F1[i] + b[i] * F2[i]
        dg = np.sqrt(np.diag(F1[i]) + np.diag(F2[i]))
        got = F[fo[i]:fo[i + 1]].reshape(n, n)
        assert np.all(np.abs(got - ref) <= 1e-9 * np.outer(dg, dg)), i
    # clearing restores the handle
    p2.set_bridge_partner(None)
    l3, g3 = lib.logl_grad_batch(p2, off, th, be)
    torch.cuda.synchronize()
    assert torch.equal(l3, plain_l) and torch.equal(g3, plain_g)
    with pytest.raises(lib.SmcxError, match="own"):
        p2.set_bridge_partner(p2)


@pytest.mark.parametrize("B_own,B_partner", [(128, 128), (200, 96), (96, 200)],
                         ids=["same", "wide_own", "wide_partner"])
def test_bridge_bands_of_different_widths(lib, orc, B_own, B_partner):
    """A bridge whose two bands differ in width, also across the 128-bin
    line where the kernels go from two to four band bins per lane: the
    launch is sized for the wider band and reads either side's data. logL,
    gradient and birth/death against the oracle."""
    w = wl.make_gblisa(N=120, k_lo=0, k_hi=6, n_inj=4, beta="uniform", noise=False, seed=421)
    say("gblisa_bridge_widths", B_own, B_partner)
    T2, T1 = w.T_obs, w.T_obs / 2
    k2, k1 = wl.gblisa_band(T2, B_own), wl.gblisa_band(T1, B_partner)
    d2 = orc.gblisa_spectrum(w.inj, T2, k2, B_own)
    d1 = orc.gblisa_spectrum(w.inj, T1, k1, B_partner)
    p2 = lib.Problem.frequency_domain(GBLISA, dev(d2), k2, T2, w.S, w.k_max, w.N, max(w.M, 1))
    p1 = lib.Problem.frequency_domain(GBLISA, dev(d1), k1, T1, w.S, w.k_max, w.N, max(w.M, 1))
    p2.set_bridge_partner(p1)
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    l, g = lib.logl_grad_batch(p2, off, th, be)
    tb, di = w.extra["theta_birth"], w.extra["death_idx"]
    db, dd = lib.delta_logl_birth_death(p2, off, th, be, dev(tb), dev(di))
    torch.cuda.synchronize()
    p2.device_status()
    l, g, db, dd = (x.cpu().numpy() for x in (l, g, db, dd))
    b = w.beta
    one = np.ones(w.N)
    r1l, r1g = orc.gblisa_logl_grad(d1, k1, T1, w.S, w.offsets, w.theta, one)
    r2l, r2g = orc.gblisa_logl_grad(d2, k2, T2, w.S, w.offsets, w.theta, one)
    assert np.all(np.abs(l - ((1 - b) * r1l + b * r2l)) <= 1e-9 * (np.abs(r1l) + np.abs(r2l)))
    rows = np.repeat(np.arange(w.N), w.K)
    rg = (1 - b[rows])[:, None] * r1g + b[rows][:, None] * r2g
    for i in range(w.N):
        a, c = w.offsets[i], w.offsets[i + 1]
        if a == c:
            continue
        scale = np.linalg.norm((np.abs(r1g[a:c]) + np.abs(r2g[a:c])) / NAT)
        assert np.linalg.norm((g[a:c] - rg[a:c]) / NAT) <= 1e-7 * scale, i
    b1, dd1 = orc.gblisa_delta(d1, k1, T1, w.S, w.offsets, w.theta, one, tb, di)
    b2, dd2 = orc.gblisa_delta(d2, k2, T2, w.S, w.offsets, w.theta, one, tb, di)
    sc = np.abs(b1) + np.abs(b2) + np.abs(dd1) + np.abs(dd2) + 1.0
    assert np.all(np.abs(db - ((1 - b) * b1 + b * b2)) <= 1e-9 * sc)
    assert np.all(np.abs(dd - ((1 - b) * dd1 + b * dd2)) <= 1e-9 * sc)


def test_block_diagonal_factor(lib, orc):
    """block = 8: the factor of the block-diagonal part of each metric block,
    which equals the oracle's full factor of that part (exact zeros between
    the blocks); in place, and with coupling entries that it ignores."""
    say("gblisa_block_factor")
    K = np.array([4, 1, 0, 10, 6])
    off = np.concatenate([[0], np.cumsum(K)])
    rng = np.random.default_rng(412)
    diag = [wl.spd_blocks([8] * int(k), seed=413 + i, spread=3.0) for i, k in enumerate(K)]
    bd = []
    for blocks in diag:
        n = 8 * len(blocks)
        m = np.zeros((n, n))
        for j, b in enumerate(blocks):
            m[8 * j:8 * j + 8, 8 * j:8 * j + 8] = b
        bd.append(m)
    coupled = []
    for m in bd:  # the same with (ignored) coupling between sources
        c = m.copy()
        mask = np.kron(np.eye(len(m) // 8), np.ones((8, 8))) == 0
        c[mask] = rng.normal(0, 1e-3, mask.sum()) * np.sqrt(np.outer(np.diag(m), np.diag(m)))[mask]
        coupled.append(0.5 * (c + c.T))
    ridge = np.array([1e-3, 1e-2, 0.5, 0.7, 0.3, 1.2, 1.2, 0.3])
    ref, status = orc.metric_factor(GBLISA, off, bd, ridge)
    assert np.all(status == 0)
    w = wl.make_gblisa(N=len(K), k_hi=int(K.max()), n_inj=1, seed=414)
    prob = lib.Problem.frequency_domain(GBLISA, dev(w.noise), w.k0, w.T_obs, w.S, int(K.max()),
                                        len(K), int(off[-1]))
    for inp in (bd, coupled):
        fo, Fp = wl.pack_blocks(inp)
        F = dev(Fp)
        W = lib.metric_factor(prob, dev(off), dev(fo), F, ridge, out=F, block=8)
        torch.cuda.synchronize()
        prob.device_status()
        Wg = W.cpu().numpy()
        for i, r in enumerate(ref):
            n = r.shape[0]
            if n == 0:
                continue
            g = Wg[fo[i]:fo[i + 1]].reshape(n, n)
            D = np.sqrt(np.diag(bd[i]) + np.tile(ridge, K[i]))
            gd, rd = g * D, r * D
            assert np.all(np.abs(gd - rd) <= 1e-10 * np.abs(rd).max(axis=1, keepdims=True)), i
            mask = np.kron(np.eye(n // 8), np.ones((8, 8))) == 0
            assert np.all(g[mask] == 0.0)
    with pytest.raises(lib.SmcxError, match="block"):
        lib.metric_factor(prob, dev(off), dev(fo), F, ridge, block=3)


def test_leapfrog_step_on_the_frequency_domain_model(lib, orc):
    """smcx_leapfrog on the GB model: drift, the frequency-domain gradient at
    the new point and the closing kick, against the step built from the
    oracle's gradients (identity metric: momenta in raw units, small eps)."""
    w = wl.make_gblisa(N=80, k_lo=0, k_hi=5, n_inj=4, beta="uniform", noise=True, seed=415)
    say("gblisa_leapfrog")
    d = _data(orc, w)
    prob = _problem(lib, w, d)
    rng = np.random.default_rng(416)
    scales = np.array([0.05 / w.T_obs, 1e-19, 0.02, 0.02, 0.02, 0.02, 0.02, 0.05])
    # raw-unit momenta sized so that one drift moves each coordinate by about
    # half its scale (the identity metric cannot balance the raw gradients,
    # whose f0 and fdot parts are 1e9 and 1e17 times the others)
    eps = 1e-17
    p0 = 0.5 * rng.standard_normal(w.theta.shape) * scales / eps
    dirs = np.where(rng.random(w.N) < 0.5, -1, 1).astype(np.int8)
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    l0, g0 = lib.logl_grad_batch(prob, off, th, be)
    q1, p1, g1, l1 = lib.leapfrog(prob, off, be, eps, th, dev(p0), g0, dir=dev(dirs))
    torch.cuda.synchronize()
    prob.device_status()
    q1, p1, l1 = q1.cpu().numpy(), p1.cpu().numpy(), l1.cpu().numpy()
    _, rg0 = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, w.offsets, w.theta, w.beta)
    rows = np.repeat(np.arange(w.N), w.K)
    e = eps * dirs[rows][:, None]
    ph = p0 + 0.5 * e * rg0
    rq = w.theta + e * ph
    rl, rg = orc.gblisa_logl_grad(d, w.k0, w.T_obs, w.S, w.offsets, rq, w.beta)
    rp = ph + 0.5 * e * rg
    # the kicks carry the gradient bound (1e-7 of the natural norm) in raw units
    gb = np.zeros_like(rg0)
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        if a < b:
            gb[a:b] = 1e-7 * np.linalg.norm(rg0[a:b] / NAT) * NAT
    assert np.all(np.abs(q1 - rq) <= 0.5 * eps * eps * gb + 1e-13 * np.abs(rq))
    assert np.all(np.abs(p1 - rp) <= eps * 2 * gb + 1e-12 * np.abs(rp))
    assert np.all(np.abs(l1 - rl) <= 1e-9 * np.abs(rl))


@pytest.mark.parametrize("model", ["fd", "pulse"])
def test_nuts_keeps_particles_beyond_k_max(lib, orc, model):
    """A particle with more components than the handle's k_max is not moved:
    status -1, its rows unchanged, the device flag raised; the others run
    (the frequency-domain NUTS walks per-doubling lists of active particles,
    which must never carry it)."""
    say("nuts_k_max", model)
    if model == "fd":
        w = wl.make_gblisa(N=40, k_lo=1, k_hi=6, n_inj=3, beta="half", noise=True, seed=431)
        d = _data(orc, w)
        big = lib.Problem.frequency_domain(GBLISA, dev(d), w.k0, w.T_obs, w.S, int(w.K.max()), w.N,
                                           w.M)
        prob = lib.Problem.frequency_domain(GBLISA, dev(d), w.k0, w.T_obs, w.S, 4, w.N, w.M)
        P = 8
    else:
        w = wl.make_config("pulse_mutate", N=40, T=1024, k_lo=1, k_hi=6, seed=432)
        d = orc.template_sum(w.model, w.inj, w.T, w.t_start, w.dt) + w.noise
        big = lib.Problem(w.model, dev(d), w.t_start, w.dt, w.sigma, int(w.K.max()), w.N, w.M)
        prob = lib.Problem(w.model, dev(d), w.t_start, w.dt, w.sigma, 4, w.N, w.M)
        P = 3
    off, th, be = dev(w.offsets), dev(w.theta), dev(w.beta)
    l0, g0 = lib.logl_grad_batch(big, off, th, be)
    lib.nuts_reserve(prob, 3)
    mom, dirs, ul, ut = wl.nuts_draws(w.N, w.M, P, 3, seed=433)
    q, l, g = th.clone(), l0.clone(), g0.clone()
    eps = 1e-3 if model == "pulse" else 0.3
    scales = np.ones(P) if model == "pulse" else np.array([0.05 / w.T_obs, 1e-19, 0.02, 0.02, 0.02,
                                                            0.02, 0.02, 0.05])
    Wb = dev(np.tile(np.diag(scales), (w.M, 1, 1)))
    _, steps, status = lib.nuts_transition(prob, off, be, eps, 3, q, l, g, dev(mom), dev(dirs),
                                           dev(ul), dev(ut), metric_blocks=Wb)
    torch.cuda.synchronize()
    with pytest.raises(lib.SmcxError, match="k_max"):
        prob.device_status()
    q, status, steps = q.cpu().numpy(), status.cpu().numpy(), steps.cpu().numpy()
    over = w.K > 4
    assert over.any() and (~over).any()
    for i in np.nonzero(over)[0]:
        a, b = w.offsets[i], w.offsets[i + 1]
        assert status[i] == -1 and steps[i] == 0
        assert np.array_equal(q[a:b], w.theta[a:b])
    assert np.all(steps[~over & (w.K > 0)] >= 1)
