"""Python binding of libsmcx (ctypes; argument marshalling only).

Every function here checks dtypes / devices / shapes, allocates outputs with
torch when the caller did not pass them, and forwards raw device pointers
and the current HIP stream to the C ABI declared in ``include/smcx.h``. All
arithmetic of the path runs in the library's kernels. There is no fallback:
if ``libsmcx.so`` is missing or cannot be loaded, importing the library
raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmcx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "smcx.h")

SMCX_OK, SMCX_EINVAL, SMCX_ENOMEM, SMCX_EDEVICE, SMCX_ECAPTURE = 0, -1, -2, -3, -4
KIND_LOGL, KIND_GRAD, KIND_DELTA = 0, 1, 2
PULSE, GBSINE, GBLISA = 0, 1, 2
N_PARAMS = {PULSE: 3, GBSINE: 4, GBLISA: 8}


class SmcxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"smcx error {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libsmcx.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, D, I, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int32
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "smcx_problem_create": [I, P, I64, D, D, D, I32, I64, I64, P, PP],
        "smcx_problem_create_fd": [I, P, I64, I64, D, D, I32, I64, I64, P, PP],
        "smcx_template_spectrum": [I, I64, P, D, I64, I64, P, P],
        "smcx_problem_destroy": [P],
        "smcx_device_status": [P, P],
        "logl_batch": [P, I64, P, I64, P, P, P, P],
        "logl_grad_batch": [P, I64, P, I64, P, P, P, P, P],
        "logl_grad_batch_masked": [P, I64, P, I64, P, P, P, P, P, P],
        "logl_grad_batch_static": [I, P, I64, D, D, D, I32, I64, P, I64, P, P, P, P, P],
        "smcx_issue_probe": [I, I32, I32, P, P, ctypes.POINTER(I64), P],
        "delta_logl_birth_death": [P, I64, P, I64, P, P, P, P, P, P, P],
        "delta_logl_birth_death_masked": [P, I64, P, I64, P, P, P, P, P, P, P, P],
        "reweight_extend": [P, I64, I64, I64, P, I64, P, D, P, P, P, P, P, P],
        "smcx_template_sum": [I, I64, P, I64, D, D, P, P],
        "smcx_plain_logl_grad": [P, I64, P, I64, P, P, P, P, P],
        "smcx_leapfrog": [P, I64, P, I64, P, D, P, P, P, P, P, P, P, P, P, P],
        "smcx_nuts_reserve": [P, I32],
        "smcx_nuts_transition": [P, I64, P, I64, P, D, I32, P, P, P, P, P, P, P, P, P, P, P, P,
                                 P, I32, P],
        "smcx_next_beta": [P, I64, P, P, D, D, P, P, P, P, P],
        "smcx_gauss_newton_metric": [P, I64, P, I64, P, P, P, I64, P, P],
        "smcx_gauss_newton_metric_masked": [P, I64, P, I64, P, P, P, P, I64, P, P],
        "smcx_gauss_newton_metric_blocks_masked": [P, I64, P, I64, P, P, P, P, P],
        "smcx_metric_factor": [P, I64, P, I64, P, I64, P, P, I32, P, P],
        "smcx_metric_factor_masked": [P, I64, P, I64, P, P, I64, P, P, I32, P, P],
        "smcx_nuts_transition_metric": [P, I64, P, I64, P, D, I32, P, P, P, P, P, P, P, P, I64, P,
                                        P, P, P, P, P, P, I32, P],
        "smcx_gauss_newton_metric_blocks": [P, I64, P, I64, P, P, P, P],
        "smcx_metric_factor_blocks": [P, I64, P, P, P, P],
        "smcx_metric_pool_blocks": [P, I64, P, P, P],
        "smcx_nuts_transition_metric_blocks": [P, I64, P, I64, P, D, I32, P, P, P, P, P, P, P, P, P,
                                               P, P, P, P, P, I32, P],
        "smcx_resample_systematic": [P, I64, P, I64, P, P, D, I64, P, P, P, P],
        "smcx_rj_apply": [P, I64, P, I64, P, P, P, P, P, P, P, I32, I32, D, I64, P, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.smcx_set_tiling.argtypes = [P, I32, I32, I64, I32]
    lib.smcx_set_tiling.restype = ctypes.c_int
    lib.smcx_get_tiling.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I64),
                                    ctypes.POINTER(I32)]
    lib.smcx_get_tiling.restype = ctypes.c_int
    lib.smcx_autotune.argtypes = [P, I32, I64, P, I64, P, P, I32, ctypes.c_char_p, P,
                                  ctypes.POINTER(I32), ctypes.POINTER(I64), ctypes.POINTER(I32),
                                  ctypes.POINTER(D)]
    lib.smcx_autotune.restype = ctypes.c_int
    lib.smcx_set_bridge_split.argtypes = [P, I64]
    lib.smcx_set_bridge_split.restype = ctypes.c_int
    lib.smcx_get_bridge_split.argtypes = [P, ctypes.POINTER(I64)]
    lib.smcx_get_bridge_split.restype = ctypes.c_int
    lib.smcx_set_bridge_partner.argtypes = [P, P]
    lib.smcx_set_bridge_partner.restype = ctypes.c_int
    lib.smcx_profile_begin.argtypes = [P, I32]
    lib.smcx_profile_begin.restype = ctypes.c_int
    lib.smcx_profile_end.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.smcx_profile_end.restype = ctypes.c_int
    lib.smcx_last_error.argtypes = []
    lib.smcx_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def header_functions() -> list:
    """Names of the functions ``include/smcx.h`` declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)


def last_error() -> str:
    return load_library().smcx_last_error().decode()


def _check(rc: int):
    if rc != SMCX_OK:
        raise SmcxError(rc, last_error())


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class Problem:
    """Owning wrapper of an ``smcx_problem`` handle (smcx_problem_create)."""

    def __init__(self, model: int, d: torch.Tensor, t_start: float, dt: float, sigma: float,
                 k_max: int, n_max: int, m_max: int, stream=None):
        lib = load_library()
        d = _dev(d, torch.float64, "d")
        self.model, self.P = int(model), N_PARAMS[int(model)]
        self.T, self.t_start, self.dt, self.sigma = int(d.numel()), float(t_start), float(dt), float(sigma)
        self.k_max, self.n_max, self.m_max = int(k_max), int(n_max), int(m_max)
        h = ctypes.c_void_p()
        _check(lib.smcx_problem_create(self.model, _ptr(d), self.T, self.t_start, self.dt, self.sigma,
                                       self.k_max, self.n_max, self.m_max, _stream(stream),
                                       ctypes.byref(h)))
        self.handle = h

    @classmethod
    def frequency_domain(cls, model: int, d, k0: int, T_obs: float, psd: float, k_max: int,
                         n_max: int, m_max: int, stream=None) -> "Problem":
        """Frequency-domain problem (smcx_problem_create_fd): d is the band
        spectrum of channels A and E, a complex [2, B] tensor (or float64
        [2, B, 2]) on the device, for bins k0 .. k0 + B - 1 of a record of
        length T_obs with constant one-sided PSD psd."""
        lib = load_library()
        if torch.is_complex(d):
            d = torch.view_as_real(d.to(torch.complex128).contiguous())
        d = _dev(d, torch.float64, "d")
        if d.dim() != 3 or d.shape[0] != 2 or d.shape[2] != 2:
            raise ValueError("d must be [2, B] complex or [2, B, 2] float64")
        self = cls.__new__(cls)
        self.model, self.P = int(model), N_PARAMS[int(model)]
        self.T, self.t_start, self.dt, self.sigma = 1, 0.0, 1.0, 1.0
        self.k0, self.B, self.T_obs, self.psd = int(k0), int(d.shape[1]), float(T_obs), float(psd)
        self.k_max, self.n_max, self.m_max = int(k_max), int(n_max), int(m_max)
        h = ctypes.c_void_p()
        _check(lib.smcx_problem_create_fd(self.model, _ptr(d), self.k0, self.B, self.T_obs, self.psd,
                                          self.k_max, self.n_max, self.m_max, _stream(stream),
                                          ctypes.byref(h)))
        self.handle = h
        return self

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().smcx_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_status(self, stream=None) -> None:
        _check(load_library().smcx_device_status(self.handle, _stream(stream)))

    def set_tiling(self, kind: int, S: int, chunk_len: int, sorted_: int = 0) -> None:
        _check(load_library().smcx_set_tiling(self.handle, int(kind), int(S), int(chunk_len),
                                              int(sorted_)))

    def get_tiling(self, kind: int):
        """(S, chunk_len, sorted) of one call kind."""
        S, cl, so = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(load_library().smcx_get_tiling(self.handle, int(kind), ctypes.byref(S),
                                              ctypes.byref(cl), ctypes.byref(so)))
        return S.value, cl.value, so.value

    def autotune(self, kind: int, offsets, theta, beta=None, reps: int = 5, cache_path=None,
                 stream=None):
        """Time every tiling of call kind `kind` on this population and keep the fastest.

        Returns (S, chunk_len, sorted, ms per call)."""
        offsets, N, theta, beta = _pop(self, offsets, theta, beta)
        S, cl, so, ms = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
        cp = None if cache_path is None else os.fsencode(cache_path)
        _check(load_library().smcx_autotune(self.handle, int(kind), N, _ptr(offsets), theta.shape[0],
                                            _ptr(theta), _ptr(beta), int(reps), cp,
                                            _stream(stream), ctypes.byref(S), ctypes.byref(cl),
                                            ctypes.byref(so), ctypes.byref(ms)))
        return S.value, cl.value, so.value, ms.value

    def set_bridge_split(self, split: int) -> None:
        """Samples before `split` enter every tempered call untempered (the
        posterior-start bridge); 0 restores the prior bridge."""
        _check(load_library().smcx_set_bridge_split(self.handle, int(split)))

    def set_bridge_partner(self, partner: Optional["Problem"]) -> None:
        """Bridge between two frequency-domain records (smcx_set_bridge_partner):
        tempered calls on this handle evaluate (1 - beta) logL_partner + beta
        logL_self. None clears it."""
        _check(load_library().smcx_set_bridge_partner(self.handle,
                                                       partner.handle if partner else None))
        self._partner = partner

    def get_bridge_split(self) -> int:
        v = ctypes.c_int64()
        _check(load_library().smcx_get_bridge_split(self.handle, ctypes.byref(v)))
        return int(v.value)

    def profile_begin(self, max_launches: int = 4096) -> None:
        _check(load_library().smcx_profile_begin(self.handle, int(max_launches)))

    def profile_end(self):
        """(total kernel milliseconds, number of bracketed calls) since profile_begin."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(load_library().smcx_profile_end(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def _pop(prob: Problem, offsets, theta, beta):
    offsets = _dev(offsets, torch.int64, "offsets")
    N = offsets.numel() - 1
    theta = _dev(theta, torch.float64, "theta")
    if theta.dim() != 2 or theta.shape[1] != prob.P:
        raise ValueError(f"theta must be [M, {prob.P}]")
    if beta is not None:
        beta = _dev(beta, torch.float64, "beta", (N,))
    return offsets, N, theta, beta


def logl_batch(prob: Problem, offsets, theta, beta=None, logl=None, stream=None) -> torch.Tensor:
    offsets, N, theta, beta = _pop(prob, offsets, theta, beta)
    if logl is None:
        logl = torch.empty(N, dtype=torch.float64, device=theta.device)
    logl = _dev(logl, torch.float64, "logl", (N,))
    _check(load_library().logl_batch(prob.handle, N, _ptr(offsets), theta.shape[0], _ptr(theta),
                                     _ptr(beta), _ptr(logl), _stream(stream)))
    return logl


def logl_grad_batch(prob: Problem, offsets, theta, beta=None, logl=None, grad=None, stream=None,
                    want_logl=True, mask=None):
    """(logl, grad) of logl_grad_batch; with mask (uint8 [N]) only the selected
    particles are evaluated (logl_grad_batch_masked) and the other entries are
    unspecified."""
    offsets, N, theta, beta = _pop(prob, offsets, theta, beta)
    if logl is None and want_logl:
        logl = torch.empty(N, dtype=torch.float64, device=theta.device)
    if logl is not None:
        logl = _dev(logl, torch.float64, "logl", (N,))
    if grad is None:
        grad = torch.empty_like(theta)
    grad = _dev(grad, torch.float64, "grad", tuple(theta.shape))
    if mask is not None:
        mask = _dev(mask, torch.uint8, "mask", (N,))
        _check(load_library().logl_grad_batch_masked(prob.handle, N, _ptr(offsets),
                                                     theta.shape[0], _ptr(theta), _ptr(beta),
                                                     _ptr(mask), _ptr(logl), _ptr(grad),
                                                     _stream(stream)))
        return logl, grad
    _check(load_library().logl_grad_batch(prob.handle, N, _ptr(offsets), theta.shape[0],
                                          _ptr(theta), _ptr(beta), _ptr(logl), _ptr(grad),
                                          _stream(stream)))
    return logl, grad


PROBE_KINDS = {"fma_f32": 0, "mul_f32": 1, "exp_f32": 2, "sin_f32": 3, "fma_f64": 4,
               "add_u32": 5, "cvt": 6, "sin_4fma": 7, "fmac_f32": 8, "add_f32": 9,
               "mul_f64": 10, "add_f64": 11, "dpp_mov": 12, "permlane32_swap": 13,
               "alignbit": 14}


def issue_probe(kind: str, blocks: int, iters: int, inp: torch.Tensor, out: torch.Tensor,
                stream=None) -> int:
    """Launch the VALU issue-rate probe (smcx_issue_probe); returns the number of
    lane-instructions the launch issues. The caller times it on `stream`."""
    inp = _dev(inp, torch.float32, "in")
    out = _dev(out, torch.float32, "out")
    if inp.numel() < 256 or out.numel() < int(blocks) * 256:
        raise ValueError("in needs 256 entries and out blocks * 256")
    n = ctypes.c_int64()
    _check(load_library().smcx_issue_probe(PROBE_KINDS[kind], int(blocks), int(iters), _ptr(inp),
                                           _ptr(out), ctypes.byref(n), _stream(stream)))
    return int(n.value)


def logl_grad_batch_static(model: int, d, t_start: float, dt: float, sigma: float, k_max: int,
                           offsets, theta, beta=None, logl=None, grad=None, stream=None):
    """(logl, grad) of logl_grad_batch_static: the fused pass without a problem
    handle, its workspace in the library's static device scratch (nothing is
    allocated by the call; outputs are allocated here only when not passed)."""
    model = int(model)
    P = N_PARAMS[model]
    d = _dev(d, torch.float64, "d")
    offsets = _dev(offsets, torch.int64, "offsets")
    N = offsets.numel() - 1
    theta = _dev(theta, torch.float64, "theta")
    if theta.dim() != 2 or theta.shape[1] != P:
        raise ValueError(f"theta must be [M, {P}]")
    if beta is not None:
        beta = _dev(beta, torch.float64, "beta", (N,))
    if logl is None:
        logl = torch.empty(N, dtype=torch.float64, device=theta.device)
    logl = _dev(logl, torch.float64, "logl", (N,))
    if grad is None:
        grad = torch.empty_like(theta)
    grad = _dev(grad, torch.float64, "grad", tuple(theta.shape))
    _check(load_library().logl_grad_batch_static(
        model, _ptr(d), d.numel(), float(t_start), float(dt), float(sigma), int(k_max), N,
        _ptr(offsets), theta.shape[0], _ptr(theta), _ptr(beta), _ptr(logl), _ptr(grad),
        _stream(stream)))
    return logl, grad


def delta_logl_birth_death(prob: Problem, offsets, theta, beta=None, theta_birth=None,
                           death_idx=None, dlogl_birth=None, dlogl_death=None, stream=None,
                           mask=None):
    """(dlogl_birth, dlogl_death) of delta_logl_birth_death; with mask (uint8
    [N]) only the selected particles are evaluated
    (delta_logl_birth_death_masked) and the other entries are unspecified."""
    offsets, N, theta, beta = _pop(prob, offsets, theta, beta)
    dev = theta.device
    if theta_birth is not None:
        theta_birth = _dev(theta_birth, torch.float64, "theta_birth", (N, prob.P))
        if dlogl_birth is None:
            dlogl_birth = torch.empty(N, dtype=torch.float64, device=dev)
        dlogl_birth = _dev(dlogl_birth, torch.float64, "dlogl_birth", (N,))
    if death_idx is not None:
        death_idx = _dev(death_idx, torch.int32, "death_idx", (N,))
        if dlogl_death is None:
            dlogl_death = torch.empty(N, dtype=torch.float64, device=dev)
        dlogl_death = _dev(dlogl_death, torch.float64, "dlogl_death", (N,))
    if mask is not None:
        mask = _dev(mask, torch.uint8, "mask", (N,))
        _check(load_library().delta_logl_birth_death_masked(
            prob.handle, N, _ptr(offsets), theta.shape[0], _ptr(theta), _ptr(beta), _ptr(mask),
            _ptr(theta_birth), _ptr(death_idx), _ptr(dlogl_birth), _ptr(dlogl_death),
            _stream(stream)))
        return dlogl_birth, dlogl_death
    _check(load_library().delta_logl_birth_death(prob.handle, N, _ptr(offsets), theta.shape[0],
                                                 _ptr(theta), _ptr(beta), _ptr(theta_birth), _ptr(death_idx),
                                                 _ptr(dlogl_birth), _ptr(dlogl_death),
                                                 _stream(stream)))
    return dlogl_birth, dlogl_death


def logl_grad_batch_masked(prob: Problem, offsets, theta, mask, beta=None, logl=None, grad=None,
                           stream=None):
    """logl_grad_batch_masked: logl_grad_batch for the particles with mask != 0."""
    return logl_grad_batch(prob, offsets, theta, beta, logl, grad, stream, mask=mask)


def delta_logl_birth_death_masked(prob: Problem, offsets, theta, mask, beta=None,
                                  theta_birth=None, death_idx=None, dlogl_birth=None,
                                  dlogl_death=None, stream=None):
    """delta_logl_birth_death_masked: delta_logl_birth_death for the particles
    with mask != 0."""
    return delta_logl_birth_death(prob, offsets, theta, beta, theta_birth, death_idx,
                                  dlogl_birth, dlogl_death, stream, mask=mask)


def reweight_extend(prob: Problem, T1: int, T2: int, offsets, theta, delta_beta: float,
                    logw_prev=None, out=None, stream=None):
    """Returns (logl_ext, logw, w_norm, scalars[ESS, logZ increment, max logw])."""
    offsets, N, theta, _ = _pop(prob, offsets, theta, None)
    dev = theta.device
    if logw_prev is not None:
        logw_prev = _dev(logw_prev, torch.float64, "logw_prev", (N,))
    if out is None:
        out = tuple(torch.empty(n, dtype=torch.float64, device=dev) for n in (N, N, N, 3))
    le, lw, wn, sc = (_dev(t, torch.float64, nm, (n,)) for t, nm, n in
                      zip(out, ("logl_ext", "logw", "w_norm", "scalars"), (N, N, N, 3)))
    _check(load_library().reweight_extend(prob.handle, int(T1), int(T2), N, _ptr(offsets),
                                          theta.shape[0], _ptr(theta), float(delta_beta), _ptr(logw_prev),
                                          _ptr(le), _ptr(lw), _ptr(wn), _ptr(sc), _stream(stream)))
    return le, lw, wn, sc


def template_sum(model: int, theta, T: int, t_start: float, dt: float, out=None, stream=None):
    theta = _dev(theta, torch.float64, "theta")
    K = theta.shape[0] if theta.numel() else 0
    if out is None:
        out = torch.empty(T, dtype=torch.float64, device=theta.device)
    out = _dev(out, torch.float64, "out", (T,))
    _check(load_library().smcx_template_sum(int(model), K, _ptr(theta), int(T), float(t_start),
                                            float(dt), _ptr(out), _stream(stream)))
    return out


def plain_logl_grad(prob: Problem, offsets_host, theta, beta=None, logl=None, grad=None,
                    stream=None):
    """One-particle-per-launch FP64 reference form; offsets are a host array."""
    off = np.ascontiguousarray(np.asarray(offsets_host, dtype=np.int64))
    N = off.shape[0] - 1
    theta = _dev(theta, torch.float64, "theta")
    if beta is not None:
        beta = _dev(beta, torch.float64, "beta", (N,))
    if logl is None:
        logl = torch.empty(N, dtype=torch.float64, device=theta.device)
    if grad is None:
        grad = torch.empty_like(theta)
    _check(load_library().smcx_plain_logl_grad(prob.handle, N, off.ctypes.data_as(ctypes.c_void_p),
                                               theta.shape[0], _ptr(theta), _ptr(beta), _ptr(logl), _ptr(grad),
                                               _stream(stream)))
    return logl, grad


def leapfrog(prob: Problem, offsets, beta, eps: float, q, p, g, dir=None, active=None, out=None,
             stream=None):
    """One leapfrog step; returns (q', p', g', logl') (smcx_leapfrog)."""
    offsets, N, q, beta = _pop(prob, offsets, q, beta)
    p = _dev(p, torch.float64, "p", tuple(q.shape))
    g = _dev(g, torch.float64, "g", tuple(q.shape))
    if dir is not None:
        dir = _dev(dir, torch.int8, "dir", (N,))
    if active is not None:
        active = _dev(active, torch.uint8, "active", (N,))
    if out is None:
        out = (torch.empty_like(q), torch.empty_like(q), torch.empty_like(q),
               torch.empty(N, dtype=torch.float64, device=q.device))
    qo, po, go, lo = out
    _check(load_library().smcx_leapfrog(prob.handle, N, _ptr(offsets), q.shape[0], _ptr(beta),
                                        float(eps), _ptr(dir), _ptr(active), _ptr(q), _ptr(p),
                                        _ptr(g), _ptr(qo), _ptr(po), _ptr(go), _ptr(lo),
                                        _stream(stream)))
    return qo, po, go, lo


def nuts_reserve(prob: Problem, max_depth: int) -> None:
    _check(load_library().smcx_nuts_reserve(prob.handle, int(max_depth)))


def nuts_transition(prob: Problem, offsets, beta, eps: float, max_depth: int, q, logl, grad,
                    momentum, dirs, u_leaf, u_tree, prior_lo=None, prior_hi=None, use_graph=True,
                    mask=None, metric=None, metric_blocks=None, stream=None):
    """One batched NUTS transition, in place on (q, logl, grad); particles with
    mask[i] == 0 (uint8 [N], optional) are left as they are. metric = (w_offsets,
    W), for example from metric_factor, selects the mass matrix (W^T W)^{-1}
    (smcx_nuts_transition_metric); momentum is then the whitened draw.
    metric_blocks = W [M, P, P] from metric_factor_blocks selects a block-diagonal
    one (smcx_nuts_transition_metric_blocks).

    Returns (depth, steps, status) int32 tensors [N]."""
    offsets, N, q, beta = _pop(prob, offsets, q, beta)
    logl = _dev(logl, torch.float64, "logl", (N,))
    grad = _dev(grad, torch.float64, "grad", tuple(q.shape))
    momentum = _dev(momentum, torch.float64, "momentum", tuple(q.shape))
    dirs = _dev(dirs, torch.int8, "dirs", (N, max_depth))
    u_leaf = _dev(u_leaf, torch.float64, "u_leaf", (N, (1 << max_depth) - 1))
    u_tree = _dev(u_tree, torch.float64, "u_tree", (N, max_depth))
    if prior_lo is not None:
        prior_lo = _dev(prior_lo, torch.float64, "prior_lo", (prob.P,))
        prior_hi = _dev(prior_hi, torch.float64, "prior_hi", (prob.P,))
    if mask is not None:
        mask = _dev(mask, torch.uint8, "mask", (N,))
    depth = torch.empty(N, dtype=torch.int32, device=q.device)
    steps = torch.empty_like(depth)
    status = torch.empty_like(depth)
    if metric_blocks is not None:
        W = _dev(metric_blocks, torch.float64, "W", (q.shape[0], prob.P, prob.P))
        _check(load_library().smcx_nuts_transition_metric_blocks(
            prob.handle, N, _ptr(offsets), q.shape[0], _ptr(beta), float(eps), int(max_depth),
            _ptr(prior_lo), _ptr(prior_hi), _ptr(momentum), _ptr(dirs), _ptr(u_leaf),
            _ptr(u_tree), _ptr(mask), _ptr(W), _ptr(q), _ptr(logl), _ptr(grad), _ptr(depth),
            _ptr(steps), _ptr(status), 1 if use_graph else 0, _stream(stream)))
        return depth, steps, status
    if metric is not None:
        w_off = _dev(metric[0], torch.int64, "w_offsets", (N + 1,))
        W = _dev(metric[1], torch.float64, "W")
        _check(load_library().smcx_nuts_transition_metric(
            prob.handle, N, _ptr(offsets), q.shape[0], _ptr(beta), float(eps), int(max_depth),
            _ptr(prior_lo), _ptr(prior_hi), _ptr(momentum), _ptr(dirs), _ptr(u_leaf),
            _ptr(u_tree), _ptr(mask), _ptr(w_off), W.numel(), _ptr(W), _ptr(q), _ptr(logl),
            _ptr(grad), _ptr(depth), _ptr(steps), _ptr(status), 1 if use_graph else 0,
            _stream(stream)))
        return depth, steps, status
    _check(load_library().smcx_nuts_transition(
        prob.handle, N, _ptr(offsets), q.shape[0], _ptr(beta), float(eps), int(max_depth),
        _ptr(prior_lo), _ptr(prior_hi), _ptr(momentum), _ptr(dirs), _ptr(u_leaf), _ptr(u_tree),
        _ptr(mask), _ptr(q), _ptr(logl), _ptr(grad), _ptr(depth), _ptr(steps), _ptr(status),
        1 if use_graph else 0, _stream(stream)))
    return depth, steps, status


def metric_offsets(prob: Problem, offsets) -> torch.Tensor:
    """Start of each particle's (K P)^2 block in the packed metric array (device)."""
    offsets = _dev(offsets, torch.int64, "offsets")
    n = (offsets[1:] - offsets[:-1]) * prob.P
    out = torch.zeros_like(offsets)
    out[1:] = torch.cumsum(n * n, 0)
    return out


def gauss_newton_metric(prob: Problem, offsets, theta, beta=None, f_offsets=None, out=None,
                        stream=None, mask=None):
    """Gauss-Newton metric of every particle. Returns (f_offsets, F) with particle
    i's (K P) x (K P) matrix at F[f_offsets[i]:f_offsets[i+1]] (row-major). With
    mask (uint8 [N]) the particles with mask == 0 get zero matrices
    (smcx_gauss_newton_metric_masked)."""
    offsets, N, theta, beta = _pop(prob, offsets, theta, beta)
    if f_offsets is None:
        f_offsets = metric_offsets(prob, offsets)
    f_offsets = _dev(f_offsets, torch.int64, "f_offsets", (N + 1,))
    size = int(f_offsets[-1]) if N > 0 else 0
    if out is None:
        out = torch.empty(max(size, 1), dtype=torch.float64, device=theta.device)
    out = _dev(out, torch.float64, "F")
    if mask is not None:
        mask = _dev(mask, torch.uint8, "mask", (N,))
        _check(load_library().smcx_gauss_newton_metric_masked(
            prob.handle, N, _ptr(offsets), theta.shape[0], _ptr(theta), _ptr(beta), _ptr(mask),
            _ptr(f_offsets), out.numel(), _ptr(out), _stream(stream)))
        return f_offsets, out
    _check(load_library().smcx_gauss_newton_metric(prob.handle, N, _ptr(offsets), theta.shape[0],
                                                   _ptr(theta), _ptr(beta), _ptr(f_offsets),
                                                   out.numel(), _ptr(out), _stream(stream)))
    return f_offsets, out


def gauss_newton_metric_blocks(prob: Problem, offsets, theta, beta=None, out=None, stream=None,
                               mask=None):
    """The per-source (P x P) diagonal blocks of the Gauss-Newton metric
    (smcx_gauss_newton_metric_blocks). Returns F [M, P, P], the block of source
    row m at F[m]. With mask (uint8 [N]) the particles with mask == 0 get zero
    blocks (smcx_gauss_newton_metric_blocks_masked)."""
    offsets, N, theta, beta = _pop(prob, offsets, theta, beta)
    M = theta.shape[0]
    if out is None:
        out = torch.empty((max(M, 1), prob.P, prob.P), dtype=torch.float64, device=theta.device)
    out = _dev(out, torch.float64, "F")
    if out.numel() < M * prob.P * prob.P:
        raise ValueError(f"F needs {M} blocks of {prob.P} x {prob.P}")
    if mask is not None:
        mask = _dev(mask, torch.uint8, "mask", (N,))
        _check(load_library().smcx_gauss_newton_metric_blocks_masked(
            prob.handle, N, _ptr(offsets), M, _ptr(theta), _ptr(beta), _ptr(mask), _ptr(out),
            _stream(stream)))
        return out
    _check(load_library().smcx_gauss_newton_metric_blocks(prob.handle, N, _ptr(offsets), M,
                                                          _ptr(theta), _ptr(beta), _ptr(out),
                                                          _stream(stream)))
    return out


def gauss_newton_metric_masked(prob: Problem, offsets, theta, mask, beta=None, f_offsets=None,
                               out=None, stream=None):
    """smcx_gauss_newton_metric_masked: zero matrices where mask == 0."""
    return gauss_newton_metric(prob, offsets, theta, beta, f_offsets, out, stream, mask=mask)


def gauss_newton_metric_blocks_masked(prob: Problem, offsets, theta, mask, beta=None, out=None,
                                      stream=None):
    """smcx_gauss_newton_metric_blocks_masked: zero blocks where mask == 0."""
    return gauss_newton_metric_blocks(prob, offsets, theta, beta, out, stream, mask=mask)


def metric_factor_blocks(prob: Problem, F, ridge, out=None, M=None, stream=None):
    """W_m = L_m^{-1} of F_m + diag(ridge) for every P x P block
    (smcx_metric_factor_blocks); F [M, P, P], out may be F itself."""
    F = _dev(F, torch.float64, "F")
    if M is None:
        M = F.shape[0]
    if F.numel() < M * prob.P * prob.P:
        raise ValueError(f"F holds fewer than {M} blocks of {prob.P} x {prob.P}")
    if out is None:
        out = torch.empty_like(F)
    out = _dev(out, torch.float64, "W")
    if out.numel() < M * prob.P * prob.P:
        raise ValueError(f"W holds fewer than {M} blocks of {prob.P} x {prob.P}")
    r = [float(x) for x in ridge]
    if len(r) != prob.P:
        raise ValueError(f"ridge needs {prob.P} values")
    rarr = (ctypes.c_double * prob.P)(*r)
    _check(load_library().smcx_metric_factor_blocks(prob.handle, int(M), _ptr(F),
                                                    ctypes.cast(rarr, ctypes.c_void_p), _ptr(out),
                                                    _stream(stream)))
    return out


def metric_pool_blocks(prob: Problem, F, M=None, out=None, stream=None) -> torch.Tensor:
    """Mean of the first M P x P blocks of F (smcx_metric_pool_blocks): the
    population-level mass matrix of a mutation step; returns [P, P]."""
    F = _dev(F, torch.float64, "F")
    if M is None:
        M = F.shape[0]
    if F.numel() < M * prob.P * prob.P:
        raise ValueError(f"F holds fewer than {M} blocks of {prob.P} x {prob.P}")
    if out is None:
        out = torch.empty((prob.P, prob.P), dtype=torch.float64, device=F.device)
    out = _dev(out, torch.float64, "F_mean", (prob.P, prob.P))
    _check(load_library().smcx_metric_pool_blocks(prob.handle, int(M), _ptr(F), _ptr(out),
                                                  _stream(stream)))
    return out


def next_beta(prob: Problem, logl, beta_prev: float, alpha: float, logw_prev=None, beta_out=None,
              stream=None):
    """ESS choice of the next inverse temperature (root of eq. ess_target) from UNTEMPERED
    log-likelihoods. Returns (beta_out [N], logw [N], w_norm [N],
    scalars [4] = beta, ESS, log Z increment, ESS evaluations), all on the device."""
    logl = _dev(logl, torch.float64, "logl")
    N = logl.numel()
    if logw_prev is not None:
        logw_prev = _dev(logw_prev, torch.float64, "logw_prev", (N,))
    if beta_out is None:
        beta_out = torch.empty(N, dtype=torch.float64, device=logl.device)
    beta_out = _dev(beta_out, torch.float64, "beta_out", (N,))
    logw = torch.empty_like(logl)
    w = torch.empty_like(logl)
    scal = torch.empty(4, dtype=torch.float64, device=logl.device)
    _check(load_library().smcx_next_beta(prob.handle, N, _ptr(logl), _ptr(logw_prev),
                                         float(beta_prev), float(alpha), _ptr(beta_out),
                                         _ptr(logw), _ptr(w), _ptr(scal), _stream(stream)))
    return beta_out, logw, w, scal


def resample_systematic(prob: Problem, offsets, theta, w_norm, u: float, m_cap: int = None,
                        stream=None):
    """Systematic resampling. Returns (ancestors int32 [N], offsets_out int64 [N+1],
    theta_out [m_cap, P]); the new population has offsets_out[N] rows."""
    offsets, N, theta, _ = _pop(prob, offsets, theta, None)
    w_norm = _dev(w_norm, torch.float64, "w_norm", (N,))
    if m_cap is None:
        m_cap = N * prob.k_max
    anc = torch.empty(N, dtype=torch.int32, device=theta.device)
    off = torch.empty(N + 1, dtype=torch.int64, device=theta.device)
    th = torch.empty((max(int(m_cap), 1), prob.P), dtype=torch.float64, device=theta.device)
    _check(load_library().smcx_resample_systematic(prob.handle, N, _ptr(offsets), theta.shape[0],
                                                   _ptr(theta), _ptr(w_norm), float(u),
                                                   int(m_cap), _ptr(anc), _ptr(off), _ptr(th),
                                                   _stream(stream)))
    return anc, off, th


def rj_apply(prob: Problem, offsets, theta, move, theta_birth, death_idx, dlogl_birth, dlogl_death,
             log_u, k_lo: int, k_hi: int, log_pd_over_pb: float = 0.0, m_cap: int = None,
             stream=None):
    """Accept/reject birth and death moves. Returns (accepted int8 [N],
    offsets_out int64 [N+1], theta_out [m_cap, P])."""
    offsets, N, theta, _ = _pop(prob, offsets, theta, None)
    move = _dev(move, torch.int8, "move", (N,))
    log_u = _dev(log_u, torch.float64, "log_u", (N,))
    if theta_birth is not None:
        theta_birth = _dev(theta_birth, torch.float64, "theta_birth", (N, prob.P))
        dlogl_birth = _dev(dlogl_birth, torch.float64, "dlogl_birth", (N,))
    if death_idx is not None:
        death_idx = _dev(death_idx, torch.int32, "death_idx", (N,))
        dlogl_death = _dev(dlogl_death, torch.float64, "dlogl_death", (N,))
    if m_cap is None:
        m_cap = theta.shape[0] + N
    acc = torch.empty(N, dtype=torch.int8, device=theta.device)
    off = torch.empty(N + 1, dtype=torch.int64, device=theta.device)
    th = torch.empty((max(int(m_cap), 1), prob.P), dtype=torch.float64, device=theta.device)
    _check(load_library().smcx_rj_apply(prob.handle, N, _ptr(offsets), theta.shape[0], _ptr(theta),
                                        _ptr(move), _ptr(theta_birth), _ptr(death_idx),
                                        _ptr(dlogl_birth), _ptr(dlogl_death), _ptr(log_u),
                                        int(k_lo), int(k_hi), float(log_pd_over_pb), int(m_cap),
                                        _ptr(off), _ptr(th), _ptr(acc), _stream(stream)))
    return acc, off, th


class LogLGrad(torch.autograd.Function):
    """Tempered population log-likelihood with the hand-written adjoint.

    forward(theta [M,P], offsets [N+1], beta [N] or None, prob) -> logl [N]
    runs the fused forward + adjoint kernel once and keeps the gradient; the
    backward pass only applies the chain rule, scaling each particle's rows
    by the incoming gradient of its log-likelihood. When theta does not need
    a gradient (no_grad, or requires_grad False) only the forward kernel runs.
    """

    @staticmethod
    def forward(ctx, theta, offsets, beta, prob):
        th = theta.detach().contiguous()
        if not ctx.needs_input_grad[0]:
            return logl_batch(prob, offsets, th, beta)
        logl, grad = logl_grad_batch(prob, offsets, th, beta)
        ctx.save_for_backward(grad, offsets)
        return logl

    @staticmethod
    def backward(ctx, g_logl):
        grad, offsets = ctx.saved_tensors
        counts = offsets[1:] - offsets[:-1]
        rows = torch.repeat_interleave(g_logl.contiguous(), counts, output_size=grad.shape[0])
        return grad * rows.unsqueeze(1), None, None, None


def metric_factor(prob: Problem, offsets, f_offsets, F, ridge, out=None, M=None, block=0,
                  stream=None, mask=None):
    """Factor W = L^{-1} of F + diag(ridge) for every particle (smcx_metric_factor):
    ridge is a sequence of P values >= 0; out may be F itself (in place);
    block = b > 0 factors the block-diagonal part in b x b blocks.
    Returns W with the blocks of f_offsets (zeros above each diagonal). With mask
    (uint8 [N]) only the selected particles are factored
    (smcx_metric_factor_masked); the others' entries of out are not written."""
    offsets = _dev(offsets, torch.int64, "offsets")
    N = offsets.numel() - 1
    f_offsets = _dev(f_offsets, torch.int64, "f_offsets", (N + 1,))
    F = _dev(F, torch.float64, "F")
    if out is None:
        out = torch.empty_like(F)
    out = _dev(out, torch.float64, "W")
    r = [float(x) for x in ridge]
    if len(r) != prob.P:
        raise ValueError(f"ridge needs {prob.P} values")
    rarr = (ctypes.c_double * prob.P)(*r)
    if M is None:
        M = int(offsets[-1]) if N > 0 else 0
    if mask is not None:
        mask = _dev(mask, torch.uint8, "mask", (N,))
        _check(load_library().smcx_metric_factor_masked(
            prob.handle, N, _ptr(offsets), int(M), _ptr(mask), _ptr(f_offsets),
            min(F.numel(), out.numel()), _ptr(F), ctypes.cast(rarr, ctypes.c_void_p), int(block),
            _ptr(out), _stream(stream)))
        return out
    _check(load_library().smcx_metric_factor(prob.handle, N, _ptr(offsets), int(M), _ptr(f_offsets),
                                             min(F.numel(), out.numel()), _ptr(F),
                                             ctypes.cast(rarr, ctypes.c_void_p), int(block),
                                             _ptr(out), _stream(stream)))
    return out


def metric_factor_masked(prob: Problem, offsets, f_offsets, F, ridge, mask, out=None, M=None,
                         block=0, stream=None):
    """smcx_metric_factor_masked: the factor for the particles with mask != 0."""
    return metric_factor(prob, offsets, f_offsets, F, ridge, out, M, block, stream, mask=mask)


def template_spectrum(model: int, theta, T_obs: float, k0: int, B: int, stream=None) -> torch.Tensor:
    """Band spectrum [2, B] (complex128, device) of the sources theta [K, 8]
    (smcx_template_spectrum; a set-up call that synchronises)."""
    theta = _dev(theta, torch.float64, "theta")
    out = torch.empty((2, int(B), 2), dtype=torch.float64, device=theta.device)
    _check(load_library().smcx_template_spectrum(int(model), theta.shape[0] if theta.dim() == 2 else 0,
                                                 _ptr(theta), float(T_obs), int(k0), int(B),
                                                 _ptr(out), _stream(stream)))
    return torch.view_as_complex(out)
