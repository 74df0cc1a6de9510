"""Pins of the oracle's NUTS mass matrix: the factor of the metric and the
transition in whitened coordinates (Sec. "No-U-Turn-Sampler": momentum drawn
from N(0, M), kinetic energy r^T M^{-1} r / 2, M the Hessian of the negative
log posterior).

* The factor W = L^{-1} of M = F + diag(ridge) against numpy's Cholesky and
  inverse (a library routine), W M W^T = I, and the refusal of matrices that
  are not positive definite.
* W = I reproduces the plain transition exactly.
* Near a noise-free fit, with M the exact Hessian there, the whitened
  potential is |x|^2 / 2, so one leapfrog step must follow the unit harmonic
  oscillator's leapfrog map in closed form; a kick or drift taken with the
  wrong side of W, or a missing factor, moves the point by O(1) relative.
"""
import numpy as np
import pytest

from paper_2609_17674_amd import workloads as wl

PULSE, GB = wl.PULSE, wl.GBSINE


def _spd_blocks(rng, ns, cond_scale=True):
    out = []
    for n in ns:
        A = rng.standard_normal((n, n))
        C = A @ A.T / n + 0.5 * np.eye(n)
        s = 10.0 ** rng.uniform(-4, 4, n) if cond_scale else np.ones(n)
        out.append(C * np.outer(s, s))
    return out


@pytest.mark.parametrize("model", [PULSE, GB])
def test_factor_matches_numpy_cholesky_inverse(orc, model):
    P = orc.n_params(model)
    rng = np.random.default_rng(90 + model)
    K = np.array([2, 0, 5, 1, 9])
    off = np.concatenate([[0], np.cumsum(K)])
    F = _spd_blocks(rng, K * P)
    ridge = 10.0 ** rng.uniform(-3, 0, P)
    # the factor reads the lower triangle only: spoil the upper one
    Fu = [f + np.triu(np.full_like(f, 1e30), 1) for f in F]
    W, status = orc.metric_factor(model, off, Fu, ridge)
    assert np.all(status == 0)
    for f, w, k in zip(F, W, K):
        n = k * P
        assert w.shape == (n, n)
        if n == 0:
            continue
        M = f + np.diag(np.tile(ridge, k))
        ref = np.linalg.inv(np.linalg.cholesky(M))
        D = np.sqrt(np.diag(M))
        # compare W D (order one) row by row
        wd, rd = w * D, ref * D
        assert np.all(np.abs(wd - rd) <= 1e-10 * np.abs(rd).max(axis=1, keepdims=True))
        assert np.array_equal(np.triu(w, 1), np.zeros((n, n)))
        assert np.allclose(w @ M @ w.T, np.eye(n), rtol=0, atol=1e-9)


def test_factor_refuses_indefinite_blocks(orc):
    off = np.array([0, 1, 2, 3])
    good = np.diag([2.0, 3.0, 4.0])
    bad = good.copy()
    bad[2, 2] = -1.0
    nan = good.copy()
    nan[1, 0] = nan[0, 1] = np.nan
    W, status = orc.metric_factor(PULSE, off, [good, bad, nan], np.zeros(3))
    assert list(status) == [0, 1, 1]
    assert np.allclose(W[0], np.diag(1 / np.sqrt([2.0, 3.0, 4.0])), rtol=1e-15, atol=0)
    assert np.all(np.isnan(W[1])) and np.all(np.isnan(W[2]))
    # the ridge can make an indefinite block definite
    W, status = orc.metric_factor(PULSE, off[:3], [good, bad], np.array([0.0, 0.0, 2.0]))
    assert list(status) == [0, 0]


def _noise_free(orc, model, seed):
    if model == PULSE:
        T = 2000
        dt, t0 = 1.0 / (T - 1), 0.0
        inj = np.array([[4.0, 0.35, 0.02], [5.0, 0.62, 0.03]])
    else:
        T, dt, t0 = 1500, 15.0, 0.0
        inj = np.array([[3.0, 1.0e-3, 2e-12, 1.0], [2.0, 1.05e-3, -1e-12, 4.0]])
    d = orc.template_sum(model, inj, T, t0, dt)
    return T, dt, t0, inj, d


@pytest.mark.parametrize("model", [PULSE, GB])
def test_identity_factor_is_the_plain_transition(orc, model):
    w = wl.make_config("pulse_small" if model == PULSE else "gb_grad", N=12, T=500, k_lo=1,
                       k_hi=4, seed=94)
    d = w.noise + orc.template_sum(model, w.inj, w.T, w.t_start, w.dt)
    beta = np.full(w.N, 0.4)
    l0, g0 = orc.logl_grad(model, d, w.t_start, w.dt, w.sigma, w.offsets, w.theta, beta)
    D = 4
    mom, dirs, ul, ut = wl.nuts_draws(w.N, w.M, w.P, D, seed=95)
    eps = 2e-4 if model == PULSE else 1e-9
    ref = orc.nuts_transition(model, d, w.t_start, w.dt, w.sigma, w.offsets, beta, eps, D,
                              w.theta, l0, g0, mom, dirs, ul, ut)
    eye = [np.eye(int(k) * w.P) for k in w.K]
    got = orc.nuts_transition_metric(model, d, w.t_start, w.dt, w.sigma, w.offsets, beta, eps, D,
                                     w.theta, l0, g0, mom, dirs, ul, ut, eye)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("model", [PULSE, GB])
def test_whitened_leapfrog_is_the_unit_oscillator(orc, model):
    T, dt, t0, inj, d = _noise_free(orc, model, 96)
    sigma = 0.8
    off = np.array([0, inj.shape[0]])
    beta = np.array([1.0])
    F = orc.fisher(model, T, t0, dt, sigma, off, inj, beta)
    (W,), status = orc.metric_factor(model, off, F, np.zeros(orc.n_params(model)))
    assert status[0] == 0
    n = inj.size
    rng = np.random.default_rng(97)
    amp = 1e-4
    eps = 0.6
    for trial in range(4):
        x0 = amp * rng.standard_normal(n)
        r0 = amp * rng.standard_normal(n)
        q0 = inj.reshape(-1) + W.T @ x0          # x = L^T (q - q*), L^T^{-1} = W^T
        l0, g0 = orc.logl_grad(model, d, t0, dt, sigma, off, q0.reshape(inj.shape), beta)
        dirs = np.ones((1, 1), dtype=np.int8)
        q1, l1, g1, depth, steps, st = orc.nuts_transition_metric(
            model, d, t0, dt, sigma, off, beta, eps, 1, q0.reshape(inj.shape), l0, g0,
            r0.reshape(inj.shape), dirs, np.zeros((1, 1)), np.zeros((1, 1)), [W])
        assert steps[0] == 1 and depth[0] == 1
        # leapfrog of H = |x|^2/2 + |r|^2/2
        rh = r0 - 0.5 * eps * x0
        x1 = x0 + eps * rh
        dq = q1.reshape(-1) - inj.reshape(-1)
        ref = W.T @ x1
        assert np.linalg.norm(dq - ref) <= 1e-3 * np.linalg.norm(ref), (trial, dq, ref)
        # the new point's log-likelihood is the oscillator's potential
        assert abs(-l1[0] - 0.5 * x1 @ x1) <= 1e-3 * 0.5 * (x1 @ x1)
