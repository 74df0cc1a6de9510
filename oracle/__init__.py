"""FP64 CPU oracle for the population likelihood (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers. The product path never imports this
package. The arithmetic lives in ``smcx_oracle.c`` (plain C, double
precision, index-order sums); this module only marshals numpy arrays.

Parity status of each function (what pins it is listed in the tests under
``tests/test_oracle_*.py``):

* ``template_sum``, ``logl``: pinned by the Gaussian overlap closed form,
  the Dirichlet-kernel closed form of sinusoid products, mpmath brute force
  and the K=0 / zero-residual / scaling invariants.
* ``logl_grad``: pinned by analytic differentiation of the closed forms and
  by central finite differences of ``logl``.
* ``delta_logl_birth_death``: pinned by the exact birth/death zero sum and by
  differences of ``logl`` between the two particle states.
* ``reweight_extend``: pinned by the segment factorisation of the white-noise
  likelihood and by textbook ESS / log-sum-exp special cases.
* ``leapfrog``: pinned by time reversibility and by the O(eps^2) energy
  error of the symplectic integrator.
* ``fisher``: pinned by the Hessian at zero residual, Gaussian moment and
  bin-centred sinusoid closed forms, symmetry, semi-definiteness, beta scaling.
* ``metric_factor``: pinned by numpy's Cholesky and inverse, W M W^T = I and
  the refusal of indefinite matrices.
* ``nuts_transition_metric``: pinned by the identity factor (equal to the
  plain transition) and by the unit harmonic oscillator that a leapfrog step
  in whitened coordinates follows near a noise-free fit.
* ``nuts_transition`` / ``nuts_transition_metric`` tree building: pinned by a
  direct statement of the transition from its definition (tests/nuts_direct.py:
  the whole trajectory laid out, every aligned block summed from its own
  points, the proposal's law in closed form) for depths 1 to 6, U-turns inside
  subtrees and of the whole trajectory, divergences at the prior box, the
  proposal frequencies and the roles of the uniforms; and by an
  importance-weighted stationarity check (the transition keeps the target's
  moments). Planted mistakes in a copy of the tree code are caught.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smcx_oracle.c")
_SRC_GB = os.path.join(_HERE, "gblisa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PULSE = 0
GBSINE = 1


def _gcc(out: str, sources) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp] + list(sources) + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no FMA contraction)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_GB))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        _gcc(_LIB, [_SRC, _SRC_GB])
    return _LIB


def build_variant(out_dir: str, edits) -> str:
    """Compile a copy of the oracle with textual edits [(old, new), ...] applied
    into out_dir: each `old` must occur exactly once in the two sources
    together (smcx_oracle.c, gblisa_oracle.c) and is replaced where it
    occurs. For the tests that plant a mistake in the oracle and check that a
    pin catches it. Returns the library path; load it with bind()."""
    srcs = {_SRC: open(_SRC).read(), _SRC_GB: open(_SRC_GB).read()}
    for old, new in edits:
        where = [k for k, v in srcs.items() for _ in range(v.count(old))]
        if len(where) != 1:
            raise ValueError(f"edit target occurs {len(where)} times: {old!r}")
        srcs[where[0]] = srcs[where[0]].replace(old, new)
    paths = []
    for k, v in srcs.items():
        c_path = os.path.join(out_dir, "variant_" + os.path.basename(k))
        with open(c_path, "w") as f:
            f.write(v)
        paths.append(c_path)
    out = os.path.join(out_dir, "liboracle_variant.so")
    _gcc(out, paths)
    return out


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = bind(_LIB)
    return _lib


def bind(path: str):
    """Load an oracle library and declare its functions' argument types."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    I = ctypes.c_int
    lib.oracle_n_params.argtypes = [I]
    lib.oracle_set_threads.argtypes = [I]
    lib.oracle_set_threads.restype = None
    lib.oracle_get_threads.restype = I
    lib.oracle_template_sum.argtypes = [I, I64, P, I64, D, D, P]
    lib.oracle_logl.argtypes = [I, P, I64, D, D, D, I64, P, P, P, P]
    lib.oracle_logl_grad.argtypes = [I, P, I64, D, D, D, I64, P, P, P, P, P]
    lib.oracle_delta_logl_birth_death.argtypes = [I, P, I64, D, D, D, I64, P, P, P, P, P, P, P]
    lib.oracle_reweight_extend.argtypes = [I, P, D, D, D, I64, I64, I64, P, P, D, P, P, P, P, P]
    lib.oracle_next_beta.argtypes = [I64, P, P, D, D, P, P, P]
    lib.oracle_resample_systematic.argtypes = [I, I64, P, P, P, D, I64, P, P, P]
    lib.oracle_rj_apply.argtypes = [I, I64, P, P, P, P, P, P, P, P, ctypes.c_int32,
                                    ctypes.c_int32, D, I64, P, P, P]
    lib.oracle_leapfrog.argtypes = [I, P, I64, D, D, D, I64, P, P, P, P, D, P, P, P, P, P]
    lib.oracle_nuts_transition.argtypes = [I, P, I64, D, D, D, I64, P, P, D, I, P, P, P, P, P, P,
                                           P, P, P, P, P, P]
    lib.oracle_logl_split.argtypes = [I, P, I64, D, D, D, I64, P, P, P, I64, P]
    lib.oracle_logl_grad_split.argtypes = [I, P, I64, D, D, D, I64, P, P, P, I64, P, P]
    lib.oracle_delta_split.argtypes = [I, P, I64, D, D, D, I64, P, P, P, P, P, I64, P, P]
    lib.oracle_leapfrog_split.argtypes = [I, P, I64, D, D, D, I64, P, P, P, P, D, P, I64, P, P,
                                          P, P]
    lib.oracle_nuts_transition_split.argtypes = [I, P, I64, D, D, D, I64, P, P, D, I, P, P, P,
                                                 P, P, P, I64, P, P, P, P, P, P]
    lib.oracle_fisher.argtypes = [I, I64, D, D, D, I64, P, P, P, P, P]
    lib.oracle_fisher_split.argtypes = [I, I64, D, D, D, I64, P, P, P, I64, P, P]
    lib.oracle_nuts_transition_metric.argtypes = [I, P, I64, D, D, D, I64, P, P, D, I, P, P,
                                                  P, P, P, P, I64, P, P, P, P, P, P, P, P]
    lib.oracle_metric_factor.argtypes = [I, I64, P, P, P, P, P, P]
    lib.oracle_gblisa_tensors.argtypes = [D, P, P]
    lib.oracle_gblisa_tensors.restype = None
    lib.oracle_gblisa_positions.argtypes = [D, P]
    lib.oracle_gblisa_positions.restype = None
    lib.oracle_gblisa_response.argtypes = [D, D, D, D, P, P]
    lib.oracle_gblisa_response.restype = None
    lib.oracle_gblisa_strain.argtypes = [P, D, P]
    lib.oracle_gblisa_strain.restype = None
    lib.oracle_gblisa_spectrum.argtypes = [I64, P, D, I, I64, I64, P]
    lib.oracle_gblisa_spectrum_dft.argtypes = [I64, P, D, I64, I64, I64, P]
    lib.oracle_gblisa_logl_grad.argtypes = [P, I64, I64, D, D, I, I64, P, P, P, P, P]
    lib.oracle_gblisa_delta.argtypes = [P, I64, I64, D, D, I, I64, P, P, P, P, P, P, P]
    lib.oracle_gblisa_fisher.argtypes = [I64, I64, D, D, I, I64, P, P, P, P, P]
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int64)


def _check(rc: int, name: str):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments (code {rc})")


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def n_params(model: int) -> int:
    return int(_load().oracle_n_params(int(model)))


def template_sum(model: int, theta: np.ndarray, T: int, t_start: float, dt: float) -> np.ndarray:
    """sum_k h_k(t_s) for s = 0..T-1 (theta is [K, P])."""
    theta = _f64(theta).reshape(-1, n_params(model))
    out = np.empty(T, dtype=np.float64)
    _check(_load().oracle_template_sum(model, theta.shape[0], _p(theta), T, t_start, dt, _p(out)),
           "template_sum")
    return out


def logl(model, d, t_start, dt, sigma, offsets, theta, beta=None) -> np.ndarray:
    d, offsets, theta, beta = _f64(d), _i64(offsets), _f64(theta), _f64(beta)
    N = offsets.shape[0] - 1
    out = np.empty(N, dtype=np.float64)
    _check(_load().oracle_logl(model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets),
                               _p(theta), _p(beta), _p(out)), "logl")
    return out


def logl_grad(model, d, t_start, dt, sigma, offsets, theta, beta=None):
    d, offsets, theta, beta = _f64(d), _i64(offsets), _f64(theta), _f64(beta)
    N = offsets.shape[0] - 1
    P = n_params(model)
    out = np.empty(N, dtype=np.float64)
    grad = np.empty((int(offsets[-1]), P), dtype=np.float64)
    _check(_load().oracle_logl_grad(model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets),
                                    _p(theta), _p(beta), _p(out), _p(grad)), "logl_grad")
    return out, grad


def delta_logl_birth_death(model, d, t_start, dt, sigma, offsets, theta, beta, theta_birth,
                           death_idx):
    d, offsets, theta, beta, theta_birth = _f64(d), _i64(offsets), _f64(theta), _f64(beta), \
        _f64(theta_birth)
    death_idx = None if death_idx is None else np.ascontiguousarray(death_idx, dtype=np.int32)
    N = offsets.shape[0] - 1
    db = np.zeros(N, dtype=np.float64)
    dd = np.zeros(N, dtype=np.float64)
    _check(_load().oracle_delta_logl_birth_death(model, _p(d), d.shape[0], t_start, dt, sigma, N,
                                                 _p(offsets), _p(theta), _p(beta), _p(theta_birth),
                                                 _p(death_idx), _p(db), _p(dd)),
           "delta_logl_birth_death")
    return db, dd


def reweight_extend(model, d, t_start, dt, sigma, T1, T2, offsets, theta, delta_beta,
                    logw_prev=None):
    d, offsets, theta, logw_prev = _f64(d), _i64(offsets), _f64(theta), _f64(logw_prev)
    N = offsets.shape[0] - 1
    logl_ext = np.empty(N)
    logw = np.empty(N)
    w = np.empty(N)
    scal = np.empty(3)
    _check(_load().oracle_reweight_extend(model, _p(d), t_start, dt, sigma, T1, T2, N, _p(offsets),
                                          _p(theta), delta_beta, _p(logw_prev), _p(logl_ext),
                                          _p(logw), _p(w), _p(scal)), "reweight_extend")
    return logl_ext, logw, w, scal


def leapfrog(model, d, t_start, dt, sigma, offsets, q, p, beta, eps, active=None):
    d, offsets, q, p, beta = _f64(d), _i64(offsets), _f64(q), _f64(p), _f64(beta)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    N = offsets.shape[0] - 1
    qo = np.empty_like(q)
    po = np.empty_like(p)
    lo = np.empty(N)
    go = np.empty_like(q)
    _check(_load().oracle_leapfrog(model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets),
                                   _p(q), _p(p), _p(beta), eps, _p(act), _p(qo), _p(po), _p(lo),
                                   _p(go)), "leapfrog")
    return qo, po, lo, go


def nuts_transition(model, d, t_start, dt, sigma, offsets, beta, eps, max_depth, q, logl, grad,
                    momentum, dirs, u_leaf, u_tree, prior_lo=None, prior_hi=None):
    """One NUTS transition per particle; returns (q, logl, grad, depth, steps, status)."""
    d, offsets, beta = _f64(d), _i64(offsets), _f64(beta)
    q, logl, grad = (np.array(x, dtype=np.float64, order="C", copy=True) for x in (q, logl, grad))
    momentum, u_leaf, u_tree = _f64(momentum), _f64(u_leaf), _f64(u_tree)
    dirs = np.ascontiguousarray(dirs, dtype=np.int8)
    lo, hi = _f64(prior_lo), _f64(prior_hi)
    N = offsets.shape[0] - 1
    depth, steps, status = (np.zeros(N, dtype=np.int32) for _ in range(3))
    _check(_load().oracle_nuts_transition(model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets),
                                          _p(beta), eps, int(max_depth), _p(lo), _p(hi), _p(momentum),
                                          _p(dirs), _p(u_leaf), _p(u_tree), _p(q), _p(logl), _p(grad),
                                          _p(depth), _p(steps), _p(status)), "nuts_transition")
    return q, logl, grad, depth, steps, status


def next_beta(logl, beta_prev, alpha, logw_prev=None):
    """ESS-bisection choice of the next inverse temperature; returns
    (logw, w_norm, scalars = [beta, ESS, logZ increment, ESS evaluations])."""
    logl, logw_prev = _f64(logl), _f64(logw_prev)
    N = logl.shape[0]
    logw, w, scal = np.empty(N), np.empty(N), np.empty(4)
    _check(_load().oracle_next_beta(N, _p(logl), _p(logw_prev), beta_prev, alpha, _p(logw), _p(w),
                                    _p(scal)), "next_beta")
    return logw, w, scal


def resample_systematic(model, offsets, theta, w_norm, u, m_cap=None):
    """Systematic resampling; returns (ancestors, offsets_out, theta_out)."""
    offsets, theta, w_norm = _i64(offsets), _f64(theta), _f64(w_norm)
    N = offsets.shape[0] - 1
    P = n_params(model)
    if m_cap is None:
        m_cap = int(np.diff(offsets).max(initial=0)) * N
    anc = np.empty(N, dtype=np.int32)
    off = np.empty(N + 1, dtype=np.int64)
    th = np.empty((max(m_cap, 1), P))
    _check(_load().oracle_resample_systematic(model, N, _p(offsets), _p(theta), _p(w_norm), u, m_cap,
                                              _p(anc), _p(off), _p(th)), "resample_systematic")
    return anc, off, th[:off[-1]].copy()


def rj_apply(model, offsets, theta, move, theta_birth, death_idx, dlogl_birth, dlogl_death, log_u,
             k_lo, k_hi, log_pd_over_pb=0.0, m_cap=None):
    """Accept/reject birth and death moves; returns (accepted, offsets_out, theta_out)."""
    offsets, theta = _i64(offsets), _f64(theta)
    theta_birth, dlogl_birth, dlogl_death, log_u = (_f64(x) for x in (theta_birth, dlogl_birth,
                                                                       dlogl_death, log_u))
    move = np.ascontiguousarray(move, dtype=np.int8)
    death_idx = None if death_idx is None else np.ascontiguousarray(death_idx, dtype=np.int32)
    N = offsets.shape[0] - 1
    P = n_params(model)
    if m_cap is None:
        m_cap = int(offsets[-1]) + N
    acc = np.empty(N, dtype=np.int8)
    off = np.empty(N + 1, dtype=np.int64)
    th = np.empty((max(m_cap, 1), P))
    _check(_load().oracle_rj_apply(model, N, _p(offsets), _p(theta), _p(move), _p(theta_birth),
                                   _p(death_idx), _p(dlogl_birth), _p(dlogl_death), _p(log_u),
                                   int(k_lo), int(k_hi), float(log_pd_over_pb), m_cap, _p(off),
                                   _p(th), _p(acc)), "rj_apply")
    return acc, off, th[:off[-1]].copy()


# ---- posterior-start bridge: samples s < split untempered, s >= split tempered by beta
def logl_split(model, d, t_start, dt, sigma, offsets, theta, beta, split):
    d, offsets, theta, beta = _f64(d), _i64(offsets), _f64(theta), _f64(beta)
    N = offsets.shape[0] - 1
    out = np.empty(N)
    _check(_load().oracle_logl_split(model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets),
                                     _p(theta), _p(beta), int(split), _p(out)), "logl_split")
    return out


def logl_grad_split(model, d, t_start, dt, sigma, offsets, theta, beta, split):
    d, offsets, theta, beta = _f64(d), _i64(offsets), _f64(theta), _f64(beta)
    N = offsets.shape[0] - 1
    out = np.empty(N)
    grad = np.empty((int(offsets[-1]), n_params(model)))
    _check(_load().oracle_logl_grad_split(model, _p(d), d.shape[0], t_start, dt, sigma, N,
                                          _p(offsets), _p(theta), _p(beta), int(split), _p(out),
                                          _p(grad)), "logl_grad_split")
    return out, grad


def delta_split(model, d, t_start, dt, sigma, offsets, theta, beta, theta_birth, death_idx, split):
    d, offsets, theta, beta, theta_birth = _f64(d), _i64(offsets), _f64(theta), _f64(beta), \
        _f64(theta_birth)
    death_idx = None if death_idx is None else np.ascontiguousarray(death_idx, dtype=np.int32)
    N = offsets.shape[0] - 1
    db, dd = np.zeros(N), np.zeros(N)
    _check(_load().oracle_delta_split(model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets),
                                      _p(theta), _p(beta), _p(theta_birth), _p(death_idx),
                                      int(split), _p(db), _p(dd)), "delta_split")
    return db, dd


def leapfrog_split(model, d, t_start, dt, sigma, offsets, q, p, beta, eps, split, active=None):
    d, offsets, q, p, beta = _f64(d), _i64(offsets), _f64(q), _f64(p), _f64(beta)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    N = offsets.shape[0] - 1
    qo, po, lo, go = np.empty_like(q), np.empty_like(p), np.empty(N), np.empty_like(q)
    _check(_load().oracle_leapfrog_split(model, _p(d), d.shape[0], t_start, dt, sigma, N,
                                         _p(offsets), _p(q), _p(p), _p(beta), eps, _p(act),
                                         int(split), _p(qo), _p(po), _p(lo), _p(go)),
           "leapfrog_split")
    return qo, po, lo, go


def nuts_transition_split(model, d, t_start, dt, sigma, offsets, beta, eps, max_depth, q, logl,
                          grad, momentum, dirs, u_leaf, u_tree, split, prior_lo=None,
                          prior_hi=None):
    d, offsets, beta = _f64(d), _i64(offsets), _f64(beta)
    q, logl, grad = (np.array(x, dtype=np.float64, order="C", copy=True) for x in (q, logl, grad))
    momentum, u_leaf, u_tree = _f64(momentum), _f64(u_leaf), _f64(u_tree)
    dirs = np.ascontiguousarray(dirs, dtype=np.int8)
    lo, hi = _f64(prior_lo), _f64(prior_hi)
    N = offsets.shape[0] - 1
    depth, steps, status = (np.zeros(N, dtype=np.int32) for _ in range(3))
    _check(_load().oracle_nuts_transition_split(
        model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets), _p(beta), eps,
        int(max_depth), _p(lo), _p(hi), _p(momentum), _p(dirs), _p(u_leaf), _p(u_tree), int(split),
        _p(q), _p(logl), _p(grad), _p(depth), _p(steps), _p(status)), "nuts_transition_split")
    return q, logl, grad, depth, steps, status


def fisher_offsets(model, offsets):
    """Start of each particle's (K P)^2 block in the packed metric array."""
    P = n_params(model)
    n = np.diff(_i64(offsets)) * P
    out = np.zeros(len(n) + 1, dtype=np.int64)
    np.cumsum(n * n, out=out[1:])
    return out


def fisher(model, T, t_start, dt, sigma, offsets, theta, beta=None, split=None):
    """Gauss-Newton metric of every particle; returns a list of (K P) x (K P) arrays.
    With split given, the metric of the posterior-start bridge target."""
    offsets, theta, beta = _i64(offsets), _f64(theta), _f64(beta)
    N = offsets.shape[0] - 1
    P = n_params(model)
    fo = fisher_offsets(model, offsets)
    F = np.empty(max(int(fo[-1]), 1))
    if split is None:
        _check(_load().oracle_fisher(model, int(T), t_start, dt, sigma, N, _p(offsets), _p(theta),
                                     _p(beta), _p(fo), _p(F)), "fisher")
    else:
        _check(_load().oracle_fisher_split(model, int(T), t_start, dt, sigma, N, _p(offsets),
                                           _p(theta), _p(beta), int(split), _p(fo), _p(F)),
               "fisher_split")
    out = []
    for i in range(N):
        n = int(offsets[i + 1] - offsets[i]) * P
        out.append(F[fo[i]:fo[i] + n * n].reshape(n, n).copy())
    return out


def pack_blocks(blocks):
    """Concatenate square blocks row-major; returns (offsets, packed array)."""
    fo = np.zeros(len(blocks) + 1, dtype=np.int64)
    np.cumsum([b.size for b in blocks], out=fo[1:])
    packed = np.concatenate([np.ravel(b) for b in blocks]) if fo[-1] else np.zeros(0)
    return fo, np.ascontiguousarray(packed, dtype=np.float64)


def metric_factor(model, offsets, blocks, ridge):
    """W = L^{-1} of M = F + diag(ridge) per particle (blocks: list of (K P)^2
    arrays); returns (list of W blocks, status array)."""
    offsets = _i64(offsets)
    N = offsets.shape[0] - 1
    fo, F = pack_blocks(blocks)
    W = np.empty(max(F.size, 1))
    status = np.zeros(N, dtype=np.int32)
    ridge = _f64(np.broadcast_to(np.asarray(ridge, dtype=np.float64), (n_params(model),)))
    _check(_load().oracle_metric_factor(model, N, _p(offsets), _p(fo), _p(F), _p(ridge), _p(W),
                                        _p(status)), "metric_factor")
    return [W[fo[i]:fo[i + 1]].reshape(blocks[i].shape).copy() for i in range(N)], status


def nuts_transition_metric(model, d, t_start, dt, sigma, offsets, beta, eps, max_depth, q, logl,
                           grad, momentum, dirs, u_leaf, u_tree, w_blocks, split=0, prior_lo=None,
                           prior_hi=None):
    """NUTS transition with the mass matrix (W^T W)^{-1}; momentum is the whitened draw."""
    d, offsets, beta = _f64(d), _i64(offsets), _f64(beta)
    q, logl, grad = (np.array(x, dtype=np.float64, order="C", copy=True) for x in (q, logl, grad))
    momentum, u_leaf, u_tree = _f64(momentum), _f64(u_leaf), _f64(u_tree)
    dirs = np.ascontiguousarray(dirs, dtype=np.int8)
    lo, hi = _f64(prior_lo), _f64(prior_hi)
    N = offsets.shape[0] - 1
    wo, W = pack_blocks(w_blocks)
    W = W if W.size else np.zeros(1)
    depth, steps, status = (np.zeros(N, dtype=np.int32) for _ in range(3))
    _check(_load().oracle_nuts_transition_metric(
        model, _p(d), d.shape[0], t_start, dt, sigma, N, _p(offsets), _p(beta), eps,
        int(max_depth), _p(lo), _p(hi), _p(momentum), _p(dirs), _p(u_leaf), _p(u_tree), int(split),
        _p(wo), _p(W), _p(q), _p(logl), _p(grad), _p(depth), _p(steps), _p(status)),
        "nuts_transition_metric")
    return q, logl, grad, depth, steps, status


# ---------------------------------------------------------------- LISA GB model
GB_P = 8
GB_NS = 64  # envelope samples of the fast/slow template


def gblisa_tensors(t):
    """Detector tensors (3x3) of the A and E channels at time t."""
    DA, DE = np.empty(9), np.empty(9)
    _load().oracle_gblisa_tensors(float(t), _p(DA), _p(DE))
    return DA.reshape(3, 3), DE.reshape(3, 3)


def gblisa_positions(t):
    x = np.empty(9)
    _load().oracle_gblisa_positions(float(t), _p(x))
    return x.reshape(3, 3)


def gblisa_response(t, beta, lam, psi):
    """(F+, Fx) of the A and E channels: two arrays of 2."""
    Fp, Fx = np.empty(2), np.empty(2)
    _load().oracle_gblisa_response(float(t), float(beta), float(lam), float(psi), _p(Fp), _p(Fx))
    return Fp, Fx


def gblisa_strain(theta, t):
    """Time-domain strain (A, E) of one source at time t."""
    th, h = _f64(theta), np.empty(2)
    _load().oracle_gblisa_strain(_p(th), float(t), _p(h))
    return h


def gblisa_spectrum(theta, T_obs, k0, B, Ns=GB_NS):
    """Band spectrum [2, B] (complex) of K sources, fast/slow decomposition."""
    th = _f64(theta).reshape(-1, GB_P)
    out = np.empty((2, B, 2))
    _check(_load().oracle_gblisa_spectrum(th.shape[0], _p(th), float(T_obs), int(Ns), int(k0), int(B),
                                          _p(out)), "gblisa_spectrum")
    return out[..., 0] + 1j * out[..., 1]


def gblisa_spectrum_dft(theta, T_obs, Nt, k0, B):
    """Band spectrum [2, B] from the plain DFT of the strain sampled at Nt points."""
    th = _f64(theta).reshape(-1, GB_P)
    out = np.empty((2, B, 2))
    _check(_load().oracle_gblisa_spectrum_dft(th.shape[0], _p(th), float(T_obs), int(Nt), int(k0),
                                              int(B), _p(out)), "gblisa_spectrum_dft")
    return out[..., 0] + 1j * out[..., 1]


def _fd_data(d):
    d = np.asarray(d)
    if np.iscomplexobj(d):
        d = np.stack([d.real, d.imag], axis=-1)
    return np.ascontiguousarray(d, dtype=np.float64)


def gblisa_logl_grad(d, k0, T_obs, S, offsets, theta, beta=None, grad=True, Ns=GB_NS):
    """Tempered logL [N] (and gradient [M, 8]) of every particle; d is [2, B] complex."""
    d = _fd_data(d)
    B = d.shape[1]
    offsets, theta, beta = _i64(offsets), _f64(theta), _f64(beta)
    N = offsets.shape[0] - 1
    logl = np.empty(N)
    g = np.zeros((max(int(offsets[-1]), 0), GB_P)) if grad else None
    _check(_load().oracle_gblisa_logl_grad(_p(d), int(k0), B, float(T_obs), float(S), int(Ns), N,
                                           _p(offsets), _p(theta), _p(beta), _p(logl), _p(g)),
           "gblisa_logl_grad")
    return (logl, g) if grad else logl


def gblisa_delta(d, k0, T_obs, S, offsets, theta, beta, theta_birth, death_idx, Ns=GB_NS):
    d = _fd_data(d)
    B = d.shape[1]
    offsets, theta, beta, tb = _i64(offsets), _f64(theta), _f64(beta), _f64(theta_birth)
    di = np.ascontiguousarray(death_idx, dtype=np.int32)
    N = offsets.shape[0] - 1
    db, dd = np.empty(N), np.empty(N)
    _check(_load().oracle_gblisa_delta(_p(d), int(k0), B, float(T_obs), float(S), int(Ns), N,
                                       _p(offsets), _p(theta), _p(beta), _p(tb), _p(di), _p(db),
                                       _p(dd)), "gblisa_delta")
    return db, dd


def gblisa_fisher(k0, B, T_obs, S, offsets, theta, beta=None, Ns=GB_NS):
    """Per-source Gauss-Newton metric blocks; returns a list of (8K) x (8K) arrays."""
    offsets, theta, beta = _i64(offsets), _f64(theta), _f64(beta)
    N = offsets.shape[0] - 1
    n = np.diff(offsets) * GB_P
    fo = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(n * n, out=fo[1:])
    F = np.empty(max(int(fo[-1]), 1))
    _check(_load().oracle_gblisa_fisher(int(k0), int(B), float(T_obs), float(S), int(Ns), N,
                                        _p(offsets), _p(theta), _p(beta), _p(fo), _p(F)),
           "gblisa_fisher")
    return [F[fo[i]:fo[i + 1]].reshape(n[i], n[i]).copy() for i in range(N)]
