"""Seeded synthetic workloads for the population likelihood.

This module only draws random numbers: injection parameters, white noise,
particle populations (ragged component counts and per-component parameters
drawn from the uniform priors), tempering values and birth/death proposals.
It contains none of the likelihood arithmetic. The data vector is assembled
by the caller as ``noise + sum of injected templates``; the templates come
from whichever implementation the caller is exercising.

Workload recipes follow the paper's two toy problems:

* Gaussian pulses (Sec. "Sequence of gaussian pulses"): components with
  parameters (amplitude, centre, width) drawn from uniform priors, analysed
  in the time domain.
* Simplified Galactic binaries (Sec. "LISA Galactic binaries"): a chirping
  sinusoid per source, A' sin(2 pi f0 t + pi fdot t^2 + phi0), with the
  amplitude prior uniform in log10 A and the data rescaled by 1e21 so that
  A' = A * 1e21 is O(1).

The configurations (sizes, priors, seeds) are:

=====  =====================================================================
pulse_small   T=1000 on t in [0,1], 3 injections, N=256, K~U{0..10}, beta=1
pulse_batch   T=4096 on t in [0,1], 8 injections, N=16384, K~U{0..20},
              beta~U[0,1] per particle
gb_grad       T=2^17 at dt=15 s, 10 injections, N=4096, K~U{0..30}, beta=1
pulse_mutate  pulse_batch data, N=8192, K~U{0..20}, common beta=0.5, one
              birth (prior draw) and one death (uniform index) per particle
gb_extend     T=2^18 at dt=15 s, 20 injections, first 2^17 samples are the
              earlier segment, N=65536, K~U{0..50}
=====  =====================================================================
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PULSE = 0
GBSINE = 1
GBLISA = 2

N_PARAMS = {PULSE: 3, GBSINE: 4, GBLISA: 8}

# Uniform prior boxes, one row per parameter: (low, high).
PULSE_PRIOR = np.array([[2.0, 6.0],      # amplitude A
                        [0.1, 0.9],      # centre t0
                        [0.01, 0.05]])   # width w (a standard deviation)
GB_PRIOR = np.array([[-22.0, -21.0],     # log10 A (before the 1e21 rescale)
                     [1.000e-3, 1.010e-3],  # f0 [Hz]
                     [1e-18, 1e-16],     # fdot [Hz/s]
                     [0.0, 2.0 * np.pi]])   # phi0 [rad]
GB_RESCALE_LOG10 = 21.0

# LISA Galactic binaries in the frequency domain (Sec. "LISA Galactic
# binaries"): theta = (f0, fdot, log10 A, latitude, longitude, psi, iota,
# phi0), one year of data, channels A and E over a band of bins
# [GBLISA_K0, GBLISA_K0 + GBLISA_B) with a constant PSD. The PSD puts the
# injections' optimal SNR in 10..40 for log10 A in [-21.6, -21.0].
GBLISA_PRIOR = np.array([[0.9997e-3, 1.0007e-3],   # f0 [Hz]
                         [1e-18, 1e-16],           # fdot [Hz/s]
                         [-22.0, -20.5],           # log10 A
                         [-0.5 * np.pi, 0.5 * np.pi],  # ecliptic latitude
                         [0.0, 2.0 * np.pi],       # ecliptic longitude
                         [0.0, np.pi],             # polarisation psi
                         [0.0, np.pi],             # inclination iota
                         [0.0, 2.0 * np.pi]])      # initial phase phi0
GBLISA_T_OBS = 31557600.0
GBLISA_PSD = 3.4e4
GBLISA_K0 = 31500
GBLISA_B = 128
GBLISA_INJ_LOG10A = (-21.6, -21.0)
GBLISA_INJ_F0 = (0.9998e-3, 1.0006e-3)

CONFIG_NAMES = ("pulse_small", "pulse_batch", "gb_grad", "pulse_mutate", "gb_extend")
CONFIG_SEEDS = (101, 102, 103, 104, 105)

_BASE = {
    "pulse_small": dict(model=PULSE, T=1000, t_start=0.0, dt=1.0 / 999.0, sigma=1.0,
                        n_inj=3, N=256, k_lo=0, k_hi=10, beta="one"),
    "pulse_batch": dict(model=PULSE, T=4096, t_start=0.0, dt=1.0 / 4095.0, sigma=1.0,
                        n_inj=8, N=16384, k_lo=0, k_hi=20, beta="uniform"),
    "gb_grad": dict(model=GBSINE, T=1 << 17, t_start=0.0, dt=15.0, sigma=1.0,
                    n_inj=10, N=4096, k_lo=0, k_hi=30, beta="one"),
    "pulse_mutate": dict(model=PULSE, T=4096, t_start=0.0, dt=1.0 / 4095.0, sigma=1.0,
                         n_inj=8, N=8192, k_lo=0, k_hi=20, beta="half",
                         rj=True, eps=1e-3, max_depth=8),
    "gb_extend": dict(model=GBSINE, T=1 << 18, t_start=0.0, dt=15.0, sigma=1.0,
                      n_inj=20, N=65536, k_lo=0, k_hi=50, beta="one",
                      T1=1 << 17, T2=1 << 18),
}


@dataclass
class Workload:
    """One seeded synthetic problem instance (host arrays, FP64 / int64)."""

    name: str
    model: int
    T: int
    t_start: float
    dt: float
    sigma: float
    inj: np.ndarray            # [n_inj, P] injected component parameters
    noise: np.ndarray          # [T] white noise, N(0, sigma^2)
    offsets: np.ndarray        # [N+1] int64 prefix sums of K_i
    theta: np.ndarray          # [M, P] component parameters, CSR rows
    beta: np.ndarray           # [N] inverse temperatures
    k_max: int
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def M(self) -> int:
        return int(self.offsets[-1])

    @property
    def P(self) -> int:
        return N_PARAMS[self.model]

    @property
    def K(self) -> np.ndarray:
        return np.diff(self.offsets)


def draw_components(model: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Draw ``n`` component parameter rows from the uniform prior box.

    Pulses: (A, t0, w). Galactic binaries: (A', f0, fdot, phi0) with
    A' = 10**(log10 A + 21) and log10 A uniform.
    """
    if model == PULSE:
        u = rng.random((n, 3))
        return PULSE_PRIOR[:, 0] + u * (PULSE_PRIOR[:, 1] - PULSE_PRIOR[:, 0])
    u = rng.random((n, 4))
    raw = GB_PRIOR[:, 0] + u * (GB_PRIOR[:, 1] - GB_PRIOR[:, 0])
    out = raw.copy()
    out[:, 0] = 10.0 ** (raw[:, 0] + GB_RESCALE_LOG10)
    return out


def draw_counts(n: int, k_lo: int, k_hi: int, rng: np.random.Generator) -> np.ndarray:
    """Inclusive discrete-uniform component counts K_i in {k_lo..k_hi}."""
    return rng.integers(k_lo, k_hi + 1, size=n).astype(np.int64)


def counts_to_offsets(K: np.ndarray) -> np.ndarray:
    off = np.zeros(K.shape[0] + 1, dtype=np.int64)
    np.cumsum(K, out=off[1:])
    return off


def make_config(name_or_idx, seed: Optional[int] = None, **overrides) -> Workload:
    """Build one named workload.

    ``overrides`` may replace any size field (``T``, ``N``, ``n_inj``,
    ``k_lo``, ``k_hi``, ``T1``, ``T2``, ``beta`` mode ...) so that tests can
    run the same recipe at reduced sizes.
    """
    if isinstance(name_or_idx, int):
        name = CONFIG_NAMES[name_or_idx]
    else:
        name = name_or_idx
    cfg = dict(_BASE[name])
    if "T" in overrides and "dt" not in overrides and cfg["model"] == PULSE:
        # keep the time axis on [0, 1] as for the full-size pulse problems
        overrides["dt"] = 1.0 / (overrides["T"] - 1)
    cfg.update(overrides)
    if seed is None:
        seed = CONFIG_SEEDS[CONFIG_NAMES.index(name)]
    s_inj, s_noise, s_part, s_beta, s_rj, s_mom = np.random.SeedSequence(seed).spawn(6)
    r_inj = np.random.default_rng(s_inj)
    r_noise = np.random.default_rng(s_noise)
    r_part = np.random.default_rng(s_part)
    r_beta = np.random.default_rng(s_beta)

    model = cfg["model"]
    T = int(cfg["T"])
    inj = draw_components(model, int(cfg["n_inj"]), r_inj)
    noise = cfg["sigma"] * r_noise.standard_normal(T)
    K = draw_counts(int(cfg["N"]), int(cfg["k_lo"]), int(cfg["k_hi"]), r_part)
    offsets = counts_to_offsets(K)
    theta = draw_components(model, int(offsets[-1]), r_part)
    N = K.shape[0]
    mode = cfg["beta"]
    if mode == "one":
        beta = np.ones(N)
    elif mode == "half":
        beta = np.full(N, 0.5)
    elif mode == "uniform":
        beta = r_beta.random(N)
    else:
        beta = np.full(N, float(mode))

    extra = {"seed": seed}
    for key in ("T1", "T2", "eps", "max_depth"):
        if key in cfg:
            extra[key] = cfg[key]
    if cfg.get("rj") or overrides.get("rj"):
        r_rj = np.random.default_rng(s_rj)
        extra["theta_birth"] = draw_components(model, N, r_rj)
        u = r_rj.random(N)
        death = np.where(K > 0, np.floor(u * np.maximum(K, 1)).astype(np.int64), -1)
        extra["death_idx"] = np.minimum(death, K - 1).astype(np.int32)
        extra["momentum_rng"] = np.random.default_rng(s_mom)
    return Workload(name=name, model=model, T=T, t_start=float(cfg["t_start"]),
                    dt=float(cfg["dt"]), sigma=float(cfg["sigma"]), inj=inj, noise=noise,
                    offsets=offsets, theta=theta, beta=beta, k_max=int(cfg["k_hi"]), extra=extra)


def subsample(w: Workload, idx: np.ndarray) -> Workload:
    """Return the workload restricted to particles ``idx`` (in that order)."""
    idx = np.asarray(idx, dtype=np.int64)
    K = w.K[idx]
    off = counts_to_offsets(K)
    rows = np.concatenate([np.arange(w.offsets[i], w.offsets[i + 1]) for i in idx]) if len(idx) else \
        np.zeros(0, dtype=np.int64)
    theta = w.theta[rows].reshape(-1, w.P)
    extra = dict(w.extra)
    for key in ("theta_birth", "death_idx"):
        if key in extra:
            extra[key] = extra[key][idx]
    return Workload(name=w.name + "_sub", model=w.model, T=w.T, t_start=w.t_start, dt=w.dt,
                    sigma=w.sigma, inj=w.inj, noise=w.noise, offsets=off, theta=theta,
                    beta=w.beta[idx], k_max=w.k_max, extra=extra)


def nuts_draws(N: int, M: int, P: int, max_depth: int, seed: int):
    """Random inputs of one NUTS transition: momenta [M,P] ~ N(0,1), doubling
    directions [N,max_depth] in {-1,+1}, leaf uniforms [N, 2^max_depth - 1],
    subtree-merge uniforms [N, max_depth]."""
    rng = np.random.default_rng(seed)
    momentum = rng.standard_normal((M, P))
    dirs = np.where(rng.random((N, max_depth)) < 0.5, -1, 1).astype(np.int8)
    u_leaf = rng.random((N, (1 << max_depth) - 1))
    u_tree = rng.random((N, max_depth))
    return momentum, dirs, u_leaf, u_tree


def spd_blocks(sizes, seed: int, spread: float = 4.0):
    """Random symmetric positive-definite matrices, one per size n: C = A A^T / n
    + I/2 (A standard normal) with rows and columns scaled by 10^U[-spread,
    spread], so that the diagonal spans many orders of magnitude as a raw-unit
    metric does."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        n = int(n)
        a = rng.standard_normal((n, n))
        c = a @ a.T / max(n, 1) + 0.5 * np.eye(n)
        s = 10.0 ** rng.uniform(-spread, spread, n)
        out.append(c * np.outer(s, s))
    return out


def whitening_draws(K, scales, seed: int, mix: float = 0.3):
    """Random mass-matrix factors W = (I + R) diag(s) per particle: R strictly
    lower triangular with N(0, mix^2 / n) entries and s the per-parameter
    scales repeated over the particle's K components, so that the drift W^T r
    of a standard-normal r moves coordinate c by about s_c."""
    rng = np.random.default_rng(seed)
    scales = np.asarray(scales, dtype=np.float64)
    out = []
    for k in K:
        n = int(k) * scales.size
        r = np.tril(rng.standard_normal((n, n)), -1) * (mix / np.sqrt(max(n, 1)))
        out.append((np.eye(n) + r) * np.tile(scales, int(k))[None, :])
    return out


def pack_blocks(blocks):
    """Concatenate square blocks row-major; returns (block offsets, packed array)."""
    fo = np.zeros(len(blocks) + 1, dtype=np.int64)
    np.cumsum([b.size for b in blocks], out=fo[1:])
    packed = np.concatenate([np.ravel(b) for b in blocks]) if fo[-1] else np.zeros(0)
    return fo, np.ascontiguousarray(packed, dtype=np.float64)


@dataclass
class GBLisaWorkload:
    """A seeded LISA Galactic-binary problem: injections, frequency-domain
    noise of the two channels over the band (zero for the noise-free case
    of the paper), and a population drawn from the prior."""

    T_obs: float
    k0: int
    B: int
    S: float
    inj: np.ndarray            # [n_inj, 8]
    noise: np.ndarray          # [2, B] complex
    offsets: np.ndarray
    theta: np.ndarray          # [M, 8]
    beta: np.ndarray
    k_max: int
    extra: dict = field(default_factory=dict)

    model = GBLISA
    P = 8

    @property
    def N(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def M(self) -> int:
        return int(self.offsets[-1])

    @property
    def K(self) -> np.ndarray:
        return np.diff(self.offsets)


def draw_gblisa(n: int, rng: np.random.Generator) -> np.ndarray:
    lo, hi = GBLISA_PRIOR[:, 0], GBLISA_PRIOR[:, 1]
    return lo + rng.random((n, 8)) * (hi - lo)


def make_gblisa(N: int = 40000, k_lo: int = 1, k_hi: int = 10, n_inj: int = 10,
                beta: str = "one", noise: bool = False, seed: int = 106) -> GBLisaWorkload:
    """Injections with f0 on an equally spaced grid over GBLISA_INJ_F0 and the
    other parameters uniform (log10 A in GBLISA_INJ_LOG10A); white noise of
    PSD S in each channel when ``noise`` (each bin's real and imaginary parts
    N(0, S T_obs / 4)); a population of N particles with K ~ U{k_lo..k_hi}
    drawn from the prior box."""
    s_inj, s_noise, s_part, s_beta, s_rj, _ = np.random.SeedSequence(seed).spawn(6)
    r_inj = np.random.default_rng(s_inj)
    inj = draw_gblisa(n_inj, r_inj)
    inj[:, 0] = np.linspace(GBLISA_INJ_F0[0], GBLISA_INJ_F0[1], n_inj) if n_inj > 1 else \
        GBLISA_INJ_F0[0]
    inj[:, 2] = r_inj.uniform(GBLISA_INJ_LOG10A[0], GBLISA_INJ_LOG10A[1], n_inj)
    sd = np.sqrt(GBLISA_PSD * GBLISA_T_OBS / 4.0)
    r_noise = np.random.default_rng(s_noise)
    nz = (sd * (r_noise.standard_normal((2, GBLISA_B)) + 1j * r_noise.standard_normal((2, GBLISA_B)))
          if noise else np.zeros((2, GBLISA_B), dtype=complex))
    r_part = np.random.default_rng(s_part)
    K = draw_counts(N, k_lo, k_hi, r_part)
    offsets = counts_to_offsets(K)
    theta = draw_gblisa(int(offsets[-1]), r_part)
    r_beta = np.random.default_rng(s_beta)
    b = {"one": np.ones(N), "half": np.full(N, 0.5), "uniform": r_beta.random(N)}[beta]
    r_rj = np.random.default_rng(s_rj)
    extra = {"seed": seed, "theta_birth": draw_gblisa(N, r_rj)}
    u = r_rj.random(N)
    extra["death_idx"] = np.where(K > 0, np.minimum(np.floor(u * np.maximum(K, 1)), K - 1),
                                  -1).astype(np.int32)
    return GBLisaWorkload(T_obs=GBLISA_T_OBS, k0=GBLISA_K0, B=GBLISA_B, S=GBLISA_PSD, inj=inj,
                          noise=nz, offsets=offsets, theta=theta, beta=b, k_max=k_hi, extra=extra)


def gblisa_band(T_obs: float, B: int = GBLISA_B):
    """First bin of a band of B bins that holds the windows (carrier bin +-32)
    of every f0 of the prior box for a record of length T_obs."""
    lo = int(np.floor(GBLISA_PRIOR[0, 0] * T_obs)) - 32
    hi = int(np.floor(GBLISA_PRIOR[0, 1] * T_obs)) + 32
    if hi - lo > B:
        raise ValueError("the band is too narrow for this record length")
    return lo - (B - (hi - lo)) // 2
