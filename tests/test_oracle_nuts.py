"""Pins of the oracle NUTS transition.

Whole trajectories have no printed reference; these tests pin the parts of
the transition that reduce to something independent: a depth-1 tree is one
leapfrog step followed by an accept/reject on exp(H0 - H1), a zero
temperature gives free drift (the U-turn test can never fire on a straight
line, so the tree grows to its full depth), and particles without components
do not move.
"""
import numpy as np

from paper_2609_17674_amd import workloads as wl

PULSE = wl.PULSE


def _problem(orc, beta_val=0.3, N=40, T=400, seed=3):
    w = wl.make_config("pulse_small", N=N, T=T, k_lo=1, k_hi=3, n_inj=2, seed=seed)
    d = w.noise + orc.template_sum(PULSE, w.inj, w.T, w.t_start, w.dt)
    beta = np.full(w.N, beta_val)
    l0, g0 = orc.logl_grad(PULSE, d, w.t_start, w.dt, w.sigma, w.offsets, w.theta, beta)
    return w, d, beta, l0, g0


def test_depth_one_is_a_leapfrog_step_with_metropolis_acceptance(orc):
    w, d, beta, l0, g0 = _problem(orc)
    mom, dirs, ul, ut = wl.nuts_draws(w.N, w.M, 3, 1, seed=5)
    eps = 2e-4
    q, l, g, depth, steps, status = orc.nuts_transition(PULSE, d, w.t_start, w.dt, w.sigma, w.offsets,
                                                        beta, eps, 1, w.theta, l0, g0, mom, dirs, ul, ut)
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        sub = np.array([0, b - a])
        e = eps * dirs[i, 0]
        q1, p1, l1, g1 = orc.leapfrog(PULSE, d, w.t_start, w.dt, w.sigma, sub, w.theta[a:b], mom[a:b],
                                      beta[i:i + 1], e)
        H0 = -l0[i] + 0.5 * np.sum(mom[a:b] ** 2)
        H1 = -l1[0] + 0.5 * np.sum(p1 ** 2)
        assert steps[i] == 1
        if not H1 - H0 <= 1000:
            assert status[i] == 2 and np.array_equal(q[a:b], w.theta[a:b])
            continue
        accept = ut[i, 0] < np.exp(min(H0 - H1, 0.0))  # min(1, e^(H0-H1)) without overflow
        ref = q1 if accept else w.theta[a:b]
        assert np.allclose(q[a:b], ref, rtol=0, atol=1e-14)
        assert depth[i] == 1 and status[i] in (1, 3)


def test_zero_temperature_drifts_to_full_depth(orc):
    w, d, beta, l0, g0 = _problem(orc, beta_val=0.0)
    D = 4
    mom, dirs, ul, ut = wl.nuts_draws(w.N, w.M, 3, D, seed=6)
    eps = 1e-6  # tiny: every point stays inside the prior box
    q, l, g, depth, steps, status = orc.nuts_transition(PULSE, d, w.t_start, w.dt, w.sigma, w.offsets,
                                                        beta, eps, D, w.theta, l0, g0, mom, dirs, ul, ut,
                                                        wl.PULSE_PRIOR[:, 0], wl.PULSE_PRIOR[:, 1])
    assert np.all(status == 3) and np.all(depth == D) and np.all(steps == (1 << D) - 1)
    assert np.all(l == 0.0) and np.all(g == 0.0)
    for i in range(w.N):
        a, b = w.offsets[i], w.offsets[i + 1]
        k = (q[a:b] - w.theta[a:b]) / (eps * mom[a:b])
        kk = np.round(k[0, 0])
        assert np.allclose(k, kk, atol=1e-6) and abs(kk) <= (1 << D) - 1


def test_particles_without_components_do_not_move(orc):
    w, d, beta, l0, g0 = _problem(orc)
    K = w.K.copy()
    K[::3] = 0
    off = wl.counts_to_offsets(K)
    rows = np.concatenate([np.arange(w.offsets[i], w.offsets[i] + K[i]) for i in range(w.N)])
    th = w.theta[rows]
    l0, g0 = orc.logl_grad(PULSE, d, w.t_start, w.dt, w.sigma, off, th, beta)
    mom, dirs, ul, ut = wl.nuts_draws(w.N, len(th), 3, 3, seed=7)
    q, l, g, depth, steps, status = orc.nuts_transition(PULSE, d, w.t_start, w.dt, w.sigma, off, beta,
                                                        1e-4, 3, th, l0, g0, mom, dirs, ul, ut)
    z = K == 0
    assert np.all(status[z] == 0) and np.all(steps[z] == 0) and np.all(l[z] == l0[z])
