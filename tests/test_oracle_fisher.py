"""Pins of the oracle's Gauss-Newton metric F = (beta/sigma^2) sum_s J_s J_s^T.

Pinned by the Hessian it approximates (at zero residual the two coincide; the
Hessian comes from Richardson central differences of the pinned gradient), by
closed forms of the pulse blocks (Gaussian moment integrals, exact by Poisson
summation for interior pulses) and of the sinusoid blocks on bin-centred
frequencies, and by symmetry, positive semi-definiteness and beta scaling.
"""
import numpy as np
import pytest

from paper_2609_17674_amd import workloads as wl

PULSE, GB = wl.PULSE, wl.GBSINE


@pytest.mark.parametrize("model", [PULSE, GB])
def test_fisher_is_the_hessian_at_zero_residual(orc, model):
    T = 400 if model == PULSE else 600
    dt = 1.0 / (T - 1) if model == PULSE else 15.0
    rng = np.random.default_rng(70 + model)
    inj = wl.draw_components(model, 2, rng)
    if model == PULSE:
        inj[:, 1] = [0.35, 0.6]
    d = orc.template_sum(model, inj, T, 0.0, dt)  # noise-free: the particle fits exactly
    off = np.array([0, 2])
    beta = np.array([0.7])
    F = orc.fisher(model, T, 0.0, dt, 1.3, off, inj, beta)[0]
    n = inj.size
    if model == GB:
        Tobs = T * dt
        scale = np.tile([1.0, 1.0 / Tobs, 1.0 / Tobs ** 2, 1.0], 2)
    else:
        scale = np.tile([1.0, inj[0, 2], inj[0, 2]], 2)
    H = np.zeros((n, n))
    for j in range(n):
        def g(h):
            th = inj.copy().reshape(-1)
            th[j] += h
            return orc.logl_grad(model, d, 0.0, dt, 1.3, off, th.reshape(inj.shape), beta)[1].reshape(-1)
        h = 1e-3 * scale[j]
        d1 = (g(h) - g(-h)) / (2 * h)
        d2 = (g(h / 2) - g(-h / 2)) / h
        H[:, j] = (4 * d2 - d1) / 3  # one Richardson level
    Fs = F * np.outer(scale, scale)
    Hs = -H * np.outer(scale, scale)
    assert np.allclose(Fs, Hs, rtol=0, atol=1e-6 * np.abs(Fs).max())


def test_fisher_pulse_blocks_closed_form(orc):
    """Interior pulses, w/dt >= 3: sums over samples equal integrals / dt."""
    T = 2000
    dt = 1.0 / (T - 1)
    th = np.array([[3.0, 0.40, 0.02], [5.0, 0.47, 0.03]])
    off = np.array([0, 2])
    sigma = 0.7
    F = orc.fisher(PULSE, T, 0.0, dt, sigma, off, th, np.array([1.0]))[0] * sigma ** 2
    rp = np.sqrt(np.pi)
    for k, (A, t0, w) in enumerate(th):
        b = F[3 * k:3 * k + 3, 3 * k:3 * k + 3]
        # sum e^2 x^m = (1/dt) int exp(-x^2/w^2) x^m dx: w rp, 0, w^3 rp / 2, 0, 3 w^5 rp / 4
        ref = np.array([[w * rp, 0.0, A * rp / 2],
                        [0.0, A * A * rp / (2 * w), 0.0],
                        [A * rp / 2, 0.0, 3 * A * A * rp / (4 * w)]]) / dt
        assert np.allclose(b, ref, rtol=1e-12, atol=1e-9 * np.abs(ref).max()), (k, b, ref)
    # cross block, amplitude-amplitude entry: overlap of two unit Gaussians
    (A1, a, w1), (A2, c, w2) = th
    ov = np.sqrt(2 * np.pi) * w1 * w2 / np.sqrt(w1 ** 2 + w2 ** 2) * \
        np.exp(-(a - c) ** 2 / (2 * (w1 ** 2 + w2 ** 2))) / dt
    assert abs(F[0, 3] - ov) <= 1e-12 * ov and abs(F[3, 0] - ov) <= 1e-12 * ov


def test_fisher_sinusoid_blocks_on_bin_centred_frequencies(orc):
    T, dt = 1024, 15.0
    f0 = 40.0 / (T * dt)  # whole number of cycles over the record
    A, phi = 0.8, 0.3
    th = np.array([[A, f0, 0.0, phi]])
    F = orc.fisher(GB, T, 0.0, dt, 1.0, np.array([0, 1]), th)[0]
    assert abs(F[0, 0] - T / 2) <= 1e-9 * T            # sum sin^2
    assert abs(F[3, 3] - A * A * T / 2) <= 1e-9 * T    # sum A^2 cos^2
    assert abs(F[0, 3]) <= 1e-9 * T                    # sum A sin cos


def test_fisher_symmetric_psd_and_beta_linear(orc):
    w = wl.make_config("gb_grad", N=6, T=700, k_lo=1, k_hi=4, seed=73)
    beta = np.linspace(0.1, 1.0, w.N)
    F1 = orc.fisher(GB, w.T, w.t_start, w.dt, w.sigma, w.offsets, w.theta, np.ones(w.N))
    Fb = orc.fisher(GB, w.T, w.t_start, w.dt, w.sigma, w.offsets, w.theta, beta)
    for i, (a, b) in enumerate(zip(F1, Fb)):
        assert np.array_equal(a, a.T)
        s = np.sqrt(np.diag(a))
        assert np.linalg.eigvalsh(a / np.outer(s, s)).min() > -1e-9
        assert np.allclose(b, beta[i] * a, rtol=1e-15, atol=0)


@pytest.mark.parametrize("model", [PULSE, GB])
def test_fisher_split_is_the_sum_of_its_segments(orc, model):
    """The bridge target's metric (samples before the split untempered, later
    ones weighted by beta) equals the metric of the first segment plus beta
    times that of the second, each computed on its own time grid."""
    w = wl.make_config("pulse_small" if model == PULSE else "gb_grad", N=5, T=900, k_lo=1,
                       k_hi=4, seed=74)
    beta = np.linspace(0.15, 0.9, w.N)
    ones = np.ones(w.N)
    for split in (1, 333, 899):
        got = orc.fisher(model, w.T, w.t_start, w.dt, w.sigma, w.offsets, w.theta, beta, split=split)
        a = orc.fisher(model, split, w.t_start, w.dt, w.sigma, w.offsets, w.theta, ones)
        b = orc.fisher(model, w.T - split, w.t_start + split * w.dt, w.dt, w.sigma, w.offsets,
                       w.theta, ones)
        for i in range(w.N):
            ref = a[i] + beta[i] * b[i]
            s = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
            assert np.all(np.abs(got[i] - ref) <= 1e-12 * s), (split, i)
    # split = T is the untempered metric and split = 0 the tempered one, exactly
    full = orc.fisher(model, w.T, w.t_start, w.dt, w.sigma, w.offsets, w.theta, beta, split=w.T)
    unt = orc.fisher(model, w.T, w.t_start, w.dt, w.sigma, w.offsets, w.theta, ones)
    zero = orc.fisher(model, w.T, w.t_start, w.dt, w.sigma, w.offsets, w.theta, beta, split=0)
    tem = orc.fisher(model, w.T, w.t_start, w.dt, w.sigma, w.offsets, w.theta, beta)
    for x, y in zip(full + zero, unt + tem):
        assert np.array_equal(x, y)
