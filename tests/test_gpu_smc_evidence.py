"""The driver's evidence estimate against an independent integral.

Sec. "Sequential Monte Carlo" estimates the evidence ratio by the product of
the mean incremental weights over the tempering steps. On a problem small
enough to integrate, the estimate of a whole prior-start run must match the
evidence computed directly:

  Z = sum_k p(k) Z_k,   Z_0 = L(no components),   Z_1 = int L(theta) dtheta / V

with K uniform on {0, 1} (so the run's birth and death moves carry mass
between the two models) and theta uniform in the prior box of volume V. Z_1
is a three-dimensional integral, computed on the CPU with the oracle's
log-likelihood by defensive importance sampling (a Gaussian around the fit
with four times the Fisher covariance, mixed with the prior), whose own
standard error is far below the tolerance. Both sides drop the same constant
-(T/2) log(2 pi sigma^2) from log L.
"""
import sys

import numpy as np
import pytest
import torch

import parity as pm
from paper_2609_17674_amd import workloads as wl

pytestmark = pytest.mark.gpu
PULSE = wl.PULSE
T = 512
DT = 1.0 / (T - 1)
SIGMA = 1.0
INJ = np.array([[3.5, 0.42, 0.025]])
LO, HI = wl.PULSE_PRIOR[:, 0], wl.PULSE_PRIOR[:, 1]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _data(orc):
    noise = np.random.default_rng(4100).standard_normal(T) * SIGMA
    return noise + orc.template_sum(PULSE, INJ, T, 0.0, DT)


def reference_log_evidence(orc, d, n=400000, seed=4101):
    """log Z for K uniform on {0, 1}, and the standard error of its Z_1 part."""
    V = float(np.prod(HI - LO))
    l0 = orc.logl(PULSE, d, 0.0, DT, SIGMA, np.array([0, 0]), np.zeros((0, 3)))[0]
    off1 = np.array([0, 1])
    F = orc.fisher(PULSE, T, 0.0, DT, SIGMA, off1, INJ, np.array([1.0]))[0]
    C = 4.0 * np.linalg.inv(F)
    rng = np.random.default_rng(seed)
    from_g = rng.random(n) < 0.9
    th = np.where(from_g[:, None], rng.multivariate_normal(INJ[0], C, size=n),
                  LO + rng.random((n, 3)) * (HI - LO))
    inside = np.all((th >= LO) & (th <= HI), axis=1)
    dq = th - INJ[0]
    log_gauss = (-0.5 * np.einsum("ij,jk,ik->i", dq, np.linalg.inv(C), dq)
                 - 0.5 * np.log(np.linalg.det(2 * np.pi * C)))
    log_q = np.logaddexp(np.log(0.9) + log_gauss, np.log(0.1) - np.log(V) + np.where(inside, 0, -np.inf))
    ll = np.full(n, -np.inf)
    idx = np.nonzero(inside)[0]
    ll[idx] = orc.logl(PULSE, d, 0.0, DT, SIGMA, np.arange(len(idx) + 1), th[idx])
    lw = ll - np.log(V) - log_q
    m = np.max(lw)
    w = np.exp(lw - m)
    log_z1 = m + np.log(np.mean(w))
    rel_se = np.std(w) / np.sqrt(n) / np.mean(w)
    log_z = np.logaddexp(np.log(0.5) + l0, np.log(0.5) + log_z1)
    return float(log_z), float(rel_se)


def test_prior_start_evidence_matches_the_integral(lib, orc):
    from paper_2609_17674_amd import smc
    d = _data(orc)
    ref, rel_se = reference_log_evidence(orc, d)
    assert rel_se < 0.01
    N = 4096
    prob = lib.Problem(PULSE, pm.to_dev(d), 0.0, DT, SIGMA, 1, N, N)
    lo, hi = pm.to_dev(LO.copy()), pm.to_dev(HI.copy())
    est = []
    for seed in range(4):
        say("evidence run", seed)
        cfg = smc.SMCConfig(N=N, k_lo=0, k_hi=1, max_iters=200, seed=900 + seed, metric=True)
        res = smc.run_prior_start(prob, lo, hi, cfg)
        torch.cuda.synchronize()
        assert res.betas[-1] == 1.0
        est.append(res.log_evidence)
        k = np.array(res.k_hist[-1], dtype=float)
        print(f"[smc] seed {seed}: log Z {res.log_evidence:.3f} ({res.iterations} iterations, "
              f"K posterior {np.round(k / k.sum(), 3)})", flush=True)
    est = np.array(est)
    print(f"[smc] reference log Z {ref:.3f} (Z_1 relative s.e. {rel_se:.1e}); estimates "
          f"{np.round(est, 3)}, mean {est.mean():.3f}, spread {est.std(ddof=1):.3f}", flush=True)
    assert abs(est.mean() - ref) < 0.2, (est, ref)
    assert np.all(np.abs(est - ref) < 0.5), (est, ref)
