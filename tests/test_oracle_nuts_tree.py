"""Pins of the oracle's NUTS tree beyond one leaf (Sec. "No-U-Turn-Sampler").

The oracle builds the tree incrementally. `nuts_direct` states the same
transition from its definition (whole trajectory laid out, every aligned
block's momentum sum summed from its own points, the proposal's probability
in closed form), sharing nothing with the oracle's tree code. On a two-pulse
problem near a noise-free fit, with the mass matrix fixed at the Fisher
matrix there (so the whitened dynamics are close to a unit oscillator and
the step size sets the depth), the two must agree on:

* the tree: completed doublings, leapfrog steps taken and the stop reason,
  for step sizes that give depths 1 to 6, stops inside a subtree, U-turns of
  the whole trajectory and divergences at a prior-box wall;
* the proposal's distribution: over many transitions from the same start
  with fresh uniforms, the frequency of each trajectory point against its
  closed-form probability;
* the uniforms' roles: a leaf uniform of 0 always takes that leaf, and the
  merge of a subtree follows min(1, W_sub / W_before).

Planted mistakes in a copy of the oracle (a U-turn sign, the merge weight,
the block alignment, the leaf-uniform index, the whole-trajectory sum, the
divergence sign) must each fail at least one of these pins.
"""

import numpy as np
import pytest

import nuts_direct as nd

PULSE = 0
T = 256
DT = 1.0 / (T - 1)
SIGMA = 0.3
INJ = np.array([[4.0, 0.45, 0.03], [3.0, 0.62, 0.02]])
K, P, D = 2, 3, 6
BOX = (np.array([0.5, 0.05, 0.005]), np.array([8.0, 0.95, 0.08]))


class Problem:
    def __init__(self, orc):
        self.orc = orc
        self.d = orc.template_sum(PULSE, INJ, T, 0.0, DT)
        self.off1 = np.array([0, K])
        self.beta1 = np.array([1.0])
        F = orc.fisher(PULSE, T, 0.0, DT, SIGMA, self.off1, INJ, self.beta1)[0]
        self.F = F + 1e-6 * np.eye(K * P)
        Wl, st = orc.metric_factor(PULSE, self.off1, [F], np.full(P, 1e-6))
        assert st[0] == 0
        self.W = Wl[0]
        self.L = np.linalg.cholesky(self.F)

    def grad(self, q):
        l, g = self.orc.logl_grad(PULSE, self.d, 0.0, DT, SIGMA, self.off1, q.reshape(K, P),
                                  self.beta1)
        return float(l[0]), g.ravel()

    def inside(self, q):
        qq = q.reshape(K, P)
        return bool(np.all(qq >= BOX[0]) and np.all(qq <= BOX[1]))

    def draws(self, rng, n, scale=1.0):
        """Starts near the fit (Laplace draws), momenta, directions."""
        q0 = [INJ.ravel() + scale * np.linalg.solve(self.L.T, rng.standard_normal(K * P))
              for _ in range(n)]
        r0 = [rng.standard_normal(K * P) for _ in range(n)]
        dirs = [np.where(rng.random(D) < 0.5, -1, 1).astype(np.int8) for _ in range(n)]
        return q0, r0, dirs

    def oracle_nuts(self, q0, r0, dirs, eps, ul, ut, box=True):
        n = len(q0)
        off = np.arange(n + 1) * K
        th = np.array(q0).reshape(-1, P)
        beta = np.ones(n)
        l0, g0 = self.orc.logl_grad(PULSE, self.d, 0.0, DT, SIGMA, off, th, beta)
        lo, hi = (BOX if box else (None, None))
        return self.orc.nuts_transition_metric(
            PULSE, self.d, 0.0, DT, SIGMA, off, beta, eps, D, th, l0, g0,
            np.array(r0).reshape(-1, P), np.array(dirs, dtype=np.int8), ul, ut, [self.W] * n,
            prior_lo=lo, prior_hi=hi)

    def direct(self, q0, r0, dirs, eps):
        step = nd.leapfrog_fn(self.grad, self.W)
        return nd.build_tree(step, self.grad, q0, r0, dirs, eps, D, inside=self.inside)


def _ambiguous(tree, tol=1e-9):
    """A U-turn test too close to zero to be decided the same way by two
    summation orders."""
    return any(abs(v) < tol for v in tree.stop_values)


def check_tree_shapes(orc, n=48, seed=11):
    """Failures of the tree comparison, and the (depth, status, mid-subtree)
    cases seen."""
    pr = Problem(orc)
    rng = np.random.default_rng(seed)
    fails, seen = [], set()
    # the last step size pushes trajectories into the prior-box walls
    for eps, scale in ((0.08, 1.0), (0.2, 1.0), (0.45, 1.0), (0.9, 1.0), (1.6, 1.0), (0.9, 40.0)):
        q0, r0, dirs = pr.draws(rng, n, scale)
        keep = [i for i in range(n) if pr.inside(q0[i])]
        q0, r0, dirs = [q0[i] for i in keep], [r0[i] for i in keep], [dirs[i] for i in keep]
        ul = rng.random((len(q0), (1 << D) - 1))
        ut = rng.random((len(q0), D))
        q, l, g, depth, steps, status = pr.oracle_nuts(q0, r0, dirs, eps, ul, ut)
        for i in range(len(q0)):
            tr = pr.direct(q0[i], r0[i], dirs[i], eps)
            if _ambiguous(tr):
                continue
            got = (int(depth[i]), int(steps[i]), int(status[i]))
            want = (tr.depth, tr.steps, tr.status)
            if got != want:
                fails.append(f"eps {eps} case {i}: oracle {got}, definition {want}")
                continue
            seen.add((tr.depth, tr.status, tr.steps != (1 << tr.depth) - 1))
            pts, _ = nd.proposal_distribution(tr)
            dist = min(np.max(np.abs(p.q - q[i * K:(i + 1) * K].ravel())) for p in pts)
            if dist > 1e-9:
                fails.append(f"eps {eps} case {i}: proposal not on the accepted trajectory")
    return fails, seen


def _match(pts, q):
    dist = [np.max(np.abs(p.q - q)) for p in pts]
    j = int(np.argmin(dist))
    return j if dist[j] <= 1e-9 else -1


def check_proposal_frequencies(orc, reps=6000, seed=12):
    """Failures of the proposal frequencies against the closed-form law."""
    pr = Problem(orc)
    rng = np.random.default_rng(seed)
    fails = []
    picked = []
    for eps in (0.2, 0.45, 0.9):
        q0, r0, dirs = pr.draws(rng, 40)
        for i in range(40):
            tr = pr.direct(q0[i], r0[i], dirs[i], eps)
            if tr.depth >= 3 and not _ambiguous(tr) and tr.status != 2:
                picked.append((eps, q0[i], r0[i], dirs[i], tr))
                break
    if len(picked) < 3:
        return ["not enough deep trees to test"]
    for eps, q0, r0, dirs, tr in picked:
        pts, prob = nd.proposal_distribution(tr)
        ul = rng.random((reps, (1 << D) - 1))
        ut = rng.random((reps, D))
        q, *_ = pr.oracle_nuts([q0] * reps, [r0] * reps, [dirs] * reps, eps, ul, ut)
        counts = np.zeros(len(pts))
        for k in range(reps):
            j = _match(pts, q[k * K:(k + 1) * K].ravel())
            if j < 0:
                return [f"eps {eps}: a proposal is not a point of the trajectory"]
            counts[j] += 1
        f = counts / reps
        sd = np.sqrt(np.maximum(prob * (1 - prob), 1e-12) / reps)
        z = np.abs(f - prob) / sd
        if np.any(z > 5.0) or np.any((prob == 0) & (counts > 0)):
            fails.append(f"eps {eps} depth {tr.depth}: max z {z.max():.1f} at point "
                         f"{int(np.argmax(z))} (freq {f[np.argmax(z)]:.4f}, p {prob[np.argmax(z)]:.4f})")
    return fails


def check_uniform_roles(orc, n=40, seed=13):
    """Failures of the deterministic uniform settings."""
    pr = Problem(orc)
    rng = np.random.default_rng(seed)
    fails = []
    for eps in (0.2, 0.45, 0.9):
        q0, r0, dirs = pr.draws(rng, n)
        trees = [pr.direct(q0[i], r0[i], dirs[i], eps) for i in range(n)]
        # a leaf uniform of 0 takes that leaf, 1 - 1e-12 takes none after it
        target = rng.integers(0, 1 << 30, size=(n, D))
        ul = np.full((n, (1 << D) - 1), 1.0 - 1e-12)
        for i in range(n):
            for j in range(D):
                ul[i, (1 << j) - 1 + target[i, j] % (1 << j)] = 0.0
        for ut_val, rule in ((0.0, "always"), (1.0 - 1e-9, "when W_sub > W_before")):
            ut = np.full((n, D), ut_val)
            q, *_ = pr.oracle_nuts(q0, r0, dirs, eps, ul, ut)
            for i, tr in enumerate(trees):
                if _ambiguous(tr):
                    continue
                H0 = tr.initial.H
                expect, logW_before, skip = tr.initial, 0.0, False
                for j, sub in enumerate(tr.subtrees):
                    lw = np.array([-(p.H - H0) for p in sub])
                    t = target[i, j] % (1 << j)
                    # leaves after the target stay out unless they dominate
                    lcum = np.logaddexp.accumulate(lw)
                    if np.any(lw[t + 1:] - lcum[t + 1:] > np.log1p(-1e-9)):
                        skip = True
                    logWj = float(lcum[-1])
                    lratio = logWj - logW_before
                    if rule == "always" or lratio > np.log1p(-1e-9):
                        expect = sub[t]
                    if rule != "always" and abs(lratio) < 1e-6:
                        skip = True
                    logW_before = float(np.logaddexp(logW_before, logWj))
                if skip:
                    continue
                if np.max(np.abs(expect.q - q[i * K:(i + 1) * K].ravel())) > 1e-9:
                    fails.append(f"eps {eps} case {i}: merge rule '{rule}' took another point")
    return fails


def test_tree_shapes_match_the_definition(orc):
    fails, seen = check_tree_shapes(orc)
    assert not fails, fails[:5]
    depths = {d for d, _, _ in seen}
    statuses = {s for _, s, _ in seen}
    assert {1, 2, 3, 4, 5, 6} <= depths, depths
    assert {1, 2, 3} <= statuses, statuses
    assert any(mid for _, s, mid in seen if s == 1), "no stop inside a subtree"


def test_proposal_frequencies_match_the_closed_form(orc):
    fails = check_proposal_frequencies(orc)
    assert not fails, fails


def test_uniform_roles(orc):
    fails = check_uniform_roles(orc)
    assert not fails, fails[:5]


MUTANTS = {
    "uturn_block_sum_sign": ("double rb = rhoS[x] - ckR[(m - 1) * n + x];",
                             "double rb = rhoS[x] + ckR[(m - 1) * n + x];"),
    "uturn_test_sign": ("turn = dl <= 0.0 || dr <= 0.0;", "turn = -dl <= 0.0 || dr <= 0.0;"),
    "merge_weight_uniform": ("u_tree[i * max_depth + j] < exp(lw_sub - lw_tree)",
                             "u_tree[i * max_depth + j] < exp(lw_sub - logaddexp(lw_tree, lw_sub))"),
    "block_alignment": ("if (leaf % ((int64_t)1 << m) != 0) break;",
                        "if ((leaf + 1) % ((int64_t)1 << m) != 0) break;"),
    "leaf_uniform_index": ("u_leaf[i * nleaf + ((int64_t)1 << j) - 1 + leaf]",
                           "u_leaf[i * nleaf + leaf]"),
    "whole_trajectory_sum": ("if (dot(rhoT, pL, n) <= 0.0 || dot(rhoT, pR, n) <= 0.0)",
                             "if (dot(rhoS, pL, n) <= 0.0 || dot(rhoS, pR, n) <= 0.0)"),
    "divergence_sign": ("if (!(H - H0 <= 1000.0))", "if (!(H0 - H <= 1000.0))"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(orc, tmp_path, monkeypatch, name):
    path = orc.build_variant(str(tmp_path), [MUTANTS[name]])
    monkeypatch.setattr(orc, "_lib", orc.bind(path))
    fails, _ = check_tree_shapes(orc, n=24)
    if not fails:
        fails = check_uniform_roles(orc, n=24)
    if not fails:
        fails = check_proposal_frequencies(orc, reps=3000)
    assert fails, f"planted mistake {name} passed every pin"
