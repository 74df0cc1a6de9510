"""A direct, non-incremental statement of the NUTS transition the oracle
implements (Sec. "No-U-Turn-Sampler"; the variant is the one the oracle's
header states: doublings in given directions, multinomial sampling inside a
subtree, biased merge of a finished subtree, the generalised U-turn test on
every aligned balanced block of a subtree and on the whole trajectory,
divergence when H rises by more than 1000).

The oracle builds the tree incrementally: running momentum sums, checkpoints
of the block starts, progressive sampling driven by one uniform per leaf.
Here the same transition is written from its definition instead: the whole
trajectory is laid out first, every block's momentum sum is summed from the
block's own points, and the probability of every point being the proposal is
computed in closed form from the energies. Nothing is shared with the
oracle's tree code; the leapfrog steps themselves take the oracle's pinned
log-likelihood gradient.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Point:
    q: np.ndarray
    r: np.ndarray      # (whitened) momentum
    logl: float
    H: float


@dataclass
class Tree:
    depth: int                      # completed doublings
    steps: int                      # leapfrog steps taken
    status: int                     # 1 U-turn, 2 divergence, 3 maximum depth
    subtrees: List[List[Point]]     # accepted subtrees, each in build order
    initial: Point
    stop_values: List[float] = field(default_factory=list)  # every U-turn dot product tested


def leapfrog_fn(grad_fn: Callable[[np.ndarray], tuple], W: Optional[np.ndarray]):
    """One leapfrog step of H(q, r) = -logL(q) + |r|^2 / 2 with the mass matrix
    (W^T W)^{-1}: kick by (e/2) W g, drift by e W^T r. grad_fn(q) -> (logl, g)."""
    def step(q, r, g, e):
        Wg = g if W is None else W @ g
        rh = r + 0.5 * e * Wg
        qn = q + e * (rh if W is None else W.T @ rh)
        ln, gn = grad_fn(qn)
        Wgn = gn if W is None else W @ gn
        rn = rh + 0.5 * e * Wgn
        return qn, rn, ln, gn
    return step


def build_tree(step, grad_fn, q0, r0, dirs, eps, max_depth, inside=lambda q: True) -> Tree:
    """The transition's tree for the given doubling directions, from the
    definition: each doubling j lays out 2^j new points on side dirs[j]; the
    doubling is refused (and the transition ends) at the first point in build
    order that diverges or completes a turning block."""
    l0, g0 = grad_fn(q0)
    H0 = -l0 + 0.5 * float(r0 @ r0)
    init = Point(q0.copy(), r0.copy(), l0, H0)
    ends = {-1: (q0.copy(), r0.copy(), g0.copy()), 1: (q0.copy(), r0.copy(), g0.copy())}
    traj = [init]            # time order
    subtrees = []
    steps = 0
    values = []
    for j in range(max_depth):
        v = int(dirs[j])
        q, r, g = ends[v]
        sub = []
        for _ in range(1 << j):
            q, r, l, g = step(q, r, g, eps * v)
            H = (-l + 0.5 * float(r @ r)) if inside(q) else np.inf
            sub.append((Point(q.copy(), r.copy(), l, H), g.copy()))
        pts = [p for p, _ in sub]
        # the first failure in build order
        for n, p in enumerate(pts):
            if not (p.H - H0 <= 1000.0):
                return Tree(j, steps + n + 1, 2, subtrees, init, values)
            for m in range(1, j + 1):
                size = 1 << m
                if (n + 1) % size:
                    continue
                block = pts[n + 1 - size:n + 1]
                rho = np.sum([b.r for b in block], axis=0)
                a, b = float(rho @ block[0].r), float(rho @ block[-1].r)
                values += [a, b]
                if a <= 0.0 or b <= 0.0:
                    return Tree(j, steps + n + 1, 1, subtrees, init, values)
        steps += 1 << j
        subtrees.append(pts)
        ends[v] = (sub[-1][0].q, sub[-1][0].r, sub[-1][1])
        traj = (pts[::-1] + traj) if v < 0 else (traj + pts)
        rho = np.sum([p.r for p in traj], axis=0)
        a, b = float(rho @ traj[0].r), float(rho @ traj[-1].r)
        values += [a, b]
        if a <= 0.0 or b <= 0.0:
            return Tree(j + 1, steps, 1, subtrees, init, values)
    return Tree(max_depth, steps, 3, subtrees, init, values)


def _logsumexp(x):
    m = float(np.max(x))
    return m + float(np.log(np.sum(np.exp(x - m)))) if np.isfinite(m) else m


def proposal_distribution(tree: Tree):
    """(points, probabilities): every point of the accepted trajectory and the
    probability that it is the transition's proposal. A subtree's sample is
    multinomial in exp(-H) over its points; after subtree j is accepted, its
    sample replaces the current proposal with probability
    min(1, W_j / W_<j), W the summed exp(-H). Weights are kept as logarithms
    relative to exp(-H0)."""
    H0 = tree.initial.H
    pts = [tree.initial]
    probs = [1.0]
    logW_prev = 0.0
    for sub in tree.subtrees:
        lw = np.array([-(p.H - H0) for p in sub])
        logWj = _logsumexp(lw)
        a = float(np.exp(min(0.0, logWj - logW_prev)))
        probs = [x * (1.0 - a) for x in probs]
        pts += sub
        probs += list(a * np.exp(lw - logWj))
        logW_prev = float(np.logaddexp(logW_prev, logWj))
    return pts, np.array(probs)
