"""Does a NUTS move keep the tempered target invariant under a given rule for
its mass matrix? (Sec. "No-U-Turn-Sampler": the momentum is drawn from
N(0, M), and the mutation of step 5 of Sec. "Algorithm and implementation"
must leave the target of eq. prior_bridge invariant.)

The check is an importance-weighted stationarity test on the oracle: draw q
from a wide Gaussian around the fit, weight each draw by target / proposal
so that the weighted sample represents the target exactly, move every draw
with one oracle NUTS transition, and compare weighted moments before and
after. An invariant kernel leaves them unchanged up to Monte Carlo error
(z = weighted mean change / its standard error).

* Identity mass matrix, and a mass matrix fixed for the whole move (the
  Fisher matrix at the fit): invariant, |z| small.
* The driver's rule, one per-component Gauss-Newton block averaged over the
  population and used by every particle for the step (it depends on the
  population, not on the moving particle's own position): invariant.
* The Gauss-Newton metric taken at each particle's own position, the rule
  the driver used before: not invariant; the test shows the bias (|z| > 6).
"""
import numpy as np
import pytest

PULSE = 0
T = 256
DT = 1.0 / (T - 1)
SIGMA = 1.5
INJ = np.array([[2.0, 0.5, 0.03]])
LO = np.array([0.0, 0.2, 0.01])
HI = np.array([8.0, 0.8, 0.06])
RIDGE = 12.0 / (HI - LO) ** 2      # the prior's precision, the driver's floor
D = 5
EPS = 0.5


def _population(orc, n, seed):
    d = orc.template_sum(PULSE, INJ, T, 0.0, DT)
    off1, b1 = np.array([0, 1]), np.array([1.0])
    F0 = orc.fisher(PULSE, T, 0.0, DT, SIGMA, off1, INJ, b1)[0]
    C = 4.0 * np.linalg.inv(F0)
    rng = np.random.default_rng(seed)
    q = rng.multivariate_normal(INJ[0], C, size=n)
    q = q[np.all((q >= LO) & (q <= HI), axis=1)]
    n = len(q)
    dq = q - INJ[0]
    log_g = -0.5 * np.einsum("ij,jk,ik->i", dq, np.linalg.inv(C), dq)
    off = np.arange(n + 1)
    beta = np.ones(n)
    l0, g0 = orc.logl_grad(PULSE, d, 0.0, DT, SIGMA, off, q, beta)
    lw = l0 - log_g
    w = np.exp(lw - lw.max())
    w /= w.sum()
    draws = (rng.standard_normal((n, 3)), np.where(rng.random((n, D)) < 0.5, -1, 1).astype(np.int8),
             rng.random((n, (1 << D) - 1)), rng.random((n, D)))
    return dict(d=d, q=q, w=w, off=off, beta=beta, l0=l0, g0=g0, draws=draws, F0=F0)


def _move(orc, pop, rule):
    d, q, off, beta, l0, g0 = (pop[k] for k in ("d", "q", "off", "beta", "l0", "g0"))
    mom, dirs, ul, ut = pop["draws"]
    n = len(q)
    if rule == "identity":
        return orc.nuts_transition(PULSE, d, 0.0, DT, SIGMA, off, beta, 1.5e-3, D, q, l0, g0, mom,
                                   dirs, ul, ut, LO, HI)[0]
    if rule == "fixed":
        blocks = [pop["F0"]]
    elif rule == "pooled":
        F = orc.fisher(PULSE, T, 0.0, DT, SIGMA, off, q, beta)
        blocks = [np.mean(np.array(F), axis=0)]
    elif rule == "own_position":
        blocks = orc.fisher(PULSE, T, 0.0, DT, SIGMA, off, q, beta)
    else:
        raise ValueError(rule)
    W, st = orc.metric_factor(PULSE, np.array([0, 1] if len(blocks) == 1 else off), blocks, RIDGE)
    assert np.all(st == 0)
    Wb = W * n if len(W) == 1 else W
    return orc.nuts_transition_metric(PULSE, d, 0.0, DT, SIGMA, off, beta, EPS, D, q, l0, g0, mom,
                                      dirs, ul, ut, Wb, prior_lo=LO, prior_hi=HI)[0]


def stationarity_z(pop, q1):
    """z of the weighted mean change of A, t0, w and their squares."""
    q, w = pop["q"], pop["w"]
    z = []
    for f in (lambda x: x[:, 0], lambda x: x[:, 1], lambda x: x[:, 2],
              lambda x: x[:, 0] ** 2, lambda x: (x[:, 1] - 0.5) ** 2, lambda x: x[:, 2] ** 2):
        dlt = f(q1) - f(q)
        m = float(np.sum(w * dlt))
        se = float(np.sqrt(np.sum(w ** 2 * (dlt - m) ** 2)))
        z.append(m / se)
    return np.array(z)


@pytest.fixture(scope="module")
def pop(orc):
    p = _population(orc, 60000, seed=21)
    assert 1.0 / np.sum(p["w"] ** 2) > 10000  # effective sample size of the weighted draws
    return p


@pytest.mark.parametrize("rule", ["identity", "fixed", "pooled"])
def test_invariant_mass_matrix_rules_keep_the_target(orc, pop, rule):
    q1 = _move(orc, pop, rule)
    moved = float(np.sum(pop["w"] * np.any(q1 != pop["q"], axis=1)))
    assert moved > 0.9, moved
    z = stationarity_z(pop, q1)
    assert np.all(np.abs(z) < 4.0), z


def test_metric_at_the_particles_own_position_is_not_invariant(orc, pop):
    q1 = _move(orc, pop, "own_position")
    z = stationarity_z(pop, q1)
    assert np.max(np.abs(z)) > 6.0, z
