"""Parity metrics and fixtures shared by the GPU tests.

Tolerances (gating):
* log-likelihood: |logL - ref| <= 1e-6 |ref| per particle; a particle whose
  reference is exactly 0 (beta = 0) must be exactly 0.
* gradient: per particle, in natural coordinates g~ = g * s with
  s = (1, w_k, w_k) for pulses and (1, 1/T_obs, 1/T_obs^2, 1) for sinusoids
  (T_obs = T dt), so that the components are commensurate:
  ||g~ - g~_ref|| / ||g~_ref|| <= 1e-5 and cos(g~, g~_ref) >= 0.99999.
* birth/death: condition-scaled, |D - D_ref| <= 1e-6 beta (|<r,h>| + |h|^2/2)
  / sigma^2 (the two inner products the difference is made of).
* reweighting: logl_ext at 1e-6 relative; log-weights, normalised weights
  and ESS with the tolerance propagated from logl_ext
  (|dlogw| <= |delta_beta| |dlogl_ext|).
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2609_17674_amd import workloads as wl

LOGL_RTOL = 1e-6
GRAD_RTOL = 1e-5
GRAD_COS = 0.99999


def data_of(w: wl.Workload) -> np.ndarray:
    """noise + injected signal, the injections synthesised by the oracle."""
    return w.noise + oracle.template_sum(w.model, w.inj, w.T, w.t_start, w.dt)


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def logl_errors(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Relative error per particle; exact zeros must match exactly (inf otherwise)."""
    err = np.abs(got - ref)
    out = np.where(ref != 0, err / np.abs(np.where(ref != 0, ref, 1.0)), np.where(err == 0, 0.0, np.inf))
    return out


def natural_scale(w_model: int, theta: np.ndarray, T: int, dt: float) -> np.ndarray:
    if w_model == wl.PULSE:
        return np.column_stack([np.ones(len(theta)), theta[:, 2], theta[:, 2]])
    Tobs = T * dt
    return np.tile(np.array([1.0, 1.0 / Tobs, 1.0 / Tobs ** 2, 1.0]), (len(theta), 1))


def grad_errors(model, offsets, theta, got, ref, T, dt):
    """(normwise relative error, cosine) per particle with K > 0, natural coordinates."""
    s = natural_scale(model, theta, T, dt)
    g1, g0 = got * s, ref * s
    rel, cos = [], []
    for i in range(len(offsets) - 1):
        a, b = offsets[i], offsets[i + 1]
        if a == b:
            continue
        x, y = g1[a:b].ravel(), g0[a:b].ravel()
        ny = np.linalg.norm(y)
        if ny == 0:
            rel.append(0.0 if np.all(x == 0) else np.inf)
            cos.append(1.0)
            continue
        rel.append(np.linalg.norm(x - y) / ny)
        cos.append(float(np.dot(x, y) / (np.linalg.norm(x) * ny)) if np.linalg.norm(x) > 0 else 0.0)
    return np.array(rel), np.array(cos)


def assert_logl(got, ref, rtol=LOGL_RTOL, what="logL"):
    e = logl_errors(np.asarray(got), np.asarray(ref))
    assert np.all(e <= rtol), f"{what}: max rel err {e.max():.3e} at {int(np.argmax(e))}"
    return e


def assert_grad(model, offsets, theta, got, ref, T, dt):
    rel, cos = grad_errors(model, offsets, theta, np.asarray(got), np.asarray(ref), T, dt)
    if len(rel):
        assert np.all(rel <= GRAD_RTOL), f"grad: max rel err {rel.max():.3e} at {int(np.argmax(rel))}"
        assert np.all(cos >= GRAD_COS), f"grad: min cos {cos.min():.8f}"
    return rel, cos


def delta_scale(model, w, comp_rows, beta, sigma, delta_ref):
    """Upper bound of beta (|<r,h>| + |h|^2/2) / sigma^2 per particle.

    From D = +-beta (<r,h> - Y/2) / sigma^2 with Y = |h|^2 the oracle's
    template energy of the moved component: |<r,h>| <= |D| sigma^2 / beta
    + Y/2, so the scale is at most |D| + beta Y / sigma^2."""
    out = np.zeros(len(comp_rows))
    for i, th in enumerate(comp_rows):
        if th is None or beta[i] == 0:
            continue
        h = oracle.template_sum(model, th[None, :], w.T, w.t_start, w.dt)
        out[i] = abs(delta_ref[i]) + beta[i] * float(np.dot(h, h)) / sigma ** 2
    return out
