"""The C ABI without a GPU: symbols, host-side argument checks, layering."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def smcx():
    from paper_2609_17674_amd import build, smcx as binding
    build.build_library(force=False)
    binding.load_library()
    return binding


def test_library_exports_every_declared_function(smcx):
    names = smcx.header_functions()
    assert {"logl_batch", "logl_grad_batch", "delta_logl_birth_death", "reweight_extend",
            "smcx_problem_create", "smcx_problem_destroy", "smcx_last_error",
            "smcx_device_status"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", smcx.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(\w+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = smcx.load_library()
    for n in names:
        assert hasattr(lib, n)


def test_binding_exposes_the_abi_names(smcx):
    for n in ("logl_batch", "logl_grad_batch", "delta_logl_birth_death", "reweight_extend",
              "logl_grad_batch_masked", "delta_logl_birth_death_masked"):
        assert callable(getattr(smcx, n))


def _raw(smcx):
    return smcx.load_library()


def test_null_handle_rejected_before_launch(smcx):
    lib = _raw(smcx)
    rc = lib.logl_batch(None, 4, None, 0, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.logl_grad_batch(None, 1, None, 0, None, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL
    rc = lib.delta_logl_birth_death(None, 1, None, 0, None, None, None, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL
    rc = lib.smcx_gauss_newton_metric_masked(None, 1, None, 0, None, None, None, None, 0, None,
                                             None)
    assert rc == smcx.SMCX_EINVAL and "mask" in smcx.last_error()
    rc = lib.smcx_gauss_newton_metric_blocks_masked(None, 1, None, 0, None, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "mask" in smcx.last_error()
    rc = lib.smcx_metric_factor_masked(None, 1, None, 0, None, None, 0, None, None, 0, None, None)
    assert rc == smcx.SMCX_EINVAL and "mask" in smcx.last_error()
    rc = lib.logl_grad_batch_masked(None, 1, None, 0, None, None, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "mask" in smcx.last_error()
    rc = lib.delta_logl_birth_death_masked(None, 1, None, 0, None, None, None, None, None, None,
                                           None, None)
    assert rc == smcx.SMCX_EINVAL and "mask" in smcx.last_error()
    rc = lib.reweight_extend(None, 0, 1, 1, None, 0, None, 0.1, None, None, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL
    rc = lib.smcx_device_status(None, None)
    assert rc == smcx.SMCX_EINVAL
    assert lib.smcx_problem_destroy(None) == smcx.SMCX_OK
    rc = lib.smcx_next_beta(None, 4, None, None, 0.0, 0.9, None, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.smcx_resample_systematic(None, 4, None, 0, None, None, 0.5, 0, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.smcx_rj_apply(None, 4, None, 0, None, None, None, None, None, None, None, 1, 5, 0.0, 0,
                           None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    out = ctypes.c_void_p()
    rc = lib.smcx_problem_create_fd(2, None, 31500, 128, 3e7, 1.0, 4, 4, 16, None, ctypes.byref(out))
    assert rc == smcx.SMCX_EINVAL and "d_dev" in smcx.last_error()
    rc = lib.smcx_problem_create_fd(1, ctypes.c_void_p(0x1000), 0, 128, 3e7, 1.0, 4, 4, 16, None,
                                    ctypes.byref(out))
    assert rc == smcx.SMCX_EINVAL and "frequency-domain" in smcx.last_error()
    rc = lib.smcx_set_bridge_partner(None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.smcx_template_spectrum(2, 1, None, 3e7, 0, 128, None, None)
    assert rc == smcx.SMCX_EINVAL
    rc = lib.smcx_metric_factor(None, 4, None, 0, None, 0, None, None, 0, None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.smcx_nuts_transition_metric(None, 4, None, 0, None, 0.1, 2, None, None, None, None,
                                         None, None, None, None, 0, None, None, None, None, None,
                                         None, None, 0, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.smcx_gauss_newton_metric_blocks(None, 4, None, 0, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.smcx_metric_factor_blocks(None, 4, None, None, None, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()
    rc = lib.smcx_nuts_transition_metric_blocks(None, 4, None, 0, None, 0.1, 2, None, None, None,
                                                None, None, None, None, None, None, None, None,
                                                None, None, None, 0, None)
    assert rc == smcx.SMCX_EINVAL and "handle" in smcx.last_error()


def test_create_argument_checks(smcx):
    lib = _raw(smcx)
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail first
    cases = [
        (dict(model=7), "model"),
        (dict(d=None), "d_dev"),
        (dict(T=0), "T"),
        (dict(T=(1 << 22) + 1), "T"),
        (dict(dt=0.0), "dt"),
        (dict(dt=float("nan")), "dt"),
        (dict(sigma=-1.0), "sigma"),
        (dict(k_max=0), "k_max"),
        (dict(k_max=513), "k_max"),
        (dict(n_max=-1), "n_max"),
        (dict(m_max=-5), "m_max"),
    ]
    for ov, word in cases:
        a = dict(model=0, d=fake, T=100, t0=0.0, dt=0.01, sigma=1.0, k_max=10, n_max=10, m_max=10)
        a.update(ov)
        rc = lib.smcx_problem_create(a["model"], a["d"], a["T"], a["t0"], a["dt"], a["sigma"],
                                     a["k_max"], a["n_max"], a["m_max"], None, ctypes.byref(out))
        assert rc == smcx.SMCX_EINVAL, ov
        assert word in smcx.last_error(), (ov, smcx.last_error())
    rc = lib.smcx_problem_create(0, fake, 100, 0.0, 0.01, 1.0, 10, 10, 10, None, None)
    assert rc == smcx.SMCX_EINVAL


def test_static_entry_point_host_checks(smcx):
    """logl_grad_batch_static rejects bad arguments and sizes beyond its static
    scratch before it touches the device (no GPU is needed to see this)."""
    lib = _raw(smcx)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail first
    base = dict(model=0, d=fake, T=1000, t0=0.0, dt=1e-3, sigma=1.0, k_max=10, N=4, off=fake,
                M=8, th=fake, beta=None, logl=fake, grad=fake)

    def call(**ov):
        a = dict(base)
        a.update(ov)
        return lib.logl_grad_batch_static(a["model"], a["d"], a["T"], a["t0"], a["dt"],
                                          a["sigma"], a["k_max"], a["N"], a["off"], a["M"],
                                          a["th"], a["beta"], a["logl"], a["grad"], None)

    for ov, word in [(dict(model=2), "model"), (dict(T=0), "T"), (dict(d=None), "d is NULL"),
                     (dict(dt=0.0), "dt"), (dict(sigma=float("inf")), "sigma"),
                     (dict(k_max=0), "k_max"), (dict(N=-1), "N"), (dict(M=-1), "M"),
                     (dict(off=None), "offsets"), (dict(grad=None), "grad")]:
        assert call(**ov) == smcx.SMCX_EINVAL, ov
        assert word in smcx.last_error(), (ov, smcx.last_error())
    assert call(N=0) == smcx.SMCX_OK
    # the FP32 copy of 2^24 samples alone exceeds the scratch
    assert call(T=1 << 24) == smcx.SMCX_ENOMEM
    assert "static scratch" in smcx.last_error()
    # a population whose work list and partial sums cannot fit
    assert call(N=1 << 23, M=1 << 23) == smcx.SMCX_ENOMEM


def test_template_sum_argument_checks(smcx):
    lib = _raw(smcx)
    assert lib.smcx_template_sum(3, 1, None, 10, 0.0, 1.0, None, None) == smcx.SMCX_EINVAL
    assert lib.smcx_template_sum(0, -1, None, 10, 0.0, 1.0, None, None) == smcx.SMCX_EINVAL
    assert lib.smcx_template_sum(0, 2, None, 10, 0.0, 1.0, None, None) == smcx.SMCX_EINVAL
    assert lib.smcx_template_sum(0, 0, None, 10, 0.0, 1.0, None, None) == smcx.SMCX_EINVAL


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2609_17674_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", text.replace("oracle-free", "")), f
    src = open(os.path.join(ROOT, "oracle", "smcx_oracle.c")).read()
    assert "TEST INFRASTRUCTURE ONLY" in src
    assert "smcx_internal" not in src and "hip" not in src.lower().replace("ship", "")


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2609_17674_amd import smcx as binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        binding.load_library()
