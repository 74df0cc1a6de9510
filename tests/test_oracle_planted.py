"""Planted mistakes in the oracle: each is caught by at least one pin.

A pin that cannot fail pins nothing. Every entry below is a plausible slip in
one formula of the oracle (a dropped factor, a wrong sign, an index off by
one, a transposed operand, the wrong side of a matrix). The test compiles a
copy of the oracle with that one edit (oracle.build_variant), binds the
session's oracle module to it, and runs the CPU pin tests of the formula's
area until one of them fails. The unedited oracle passes all of them (they
run on their own elsewhere in the suite).

Groups and their pins:
* pins: the likelihood, gradient, birth/death, reweighting and leapfrog pins
  of the time-domain models (closed forms, brute force, finite differences,
  invariants; `test_oracle_pins.py`);
* metric: the Gauss-Newton metric, its factor and the whitened transition
  (`test_oracle_fisher.py`, `test_oracle_metric_nuts.py`);
* gb: the frequency-domain Galactic-binary model (`test_oracle_gblisa.py`:
  orbit, response identities, the DFT of the time-domain strain, likelihood
  invariants, Richardson differences, metric blocks);
* smc: the temperature search, the evidence increment, systematic
  resampling and the birth/death accept/reject (`test_oracle_smc.py`: the
  two-point closed form of the ESS root, scipy's log-sum-exp, the textbook
  properties of systematic resampling, the stationary distribution of K);
* split: the posterior-start bridge target (`test_oracle_split.py`: 40-digit
  brute force, its limits at split = 0 and T, birth + death = 0, depth-1
  NUTS as Metropolis on the split energy).
The NUTS tree has its own planted mistakes in `test_oracle_nuts_tree.py`.
"""
import importlib
import inspect

import pytest

GROUPS = {
    "pins": ["test_oracle_pins"],
    "metric": ["test_oracle_fisher", "test_oracle_metric_nuts"],
    "gb": ["test_oracle_gblisa"],
    "smc": ["test_oracle_smc"],
    "split": ["test_oracle_split"],
}

MUTANTS = {
    # ---------------------------------------------------------------- time-domain models
    "pulse_exponent": ("pins", "return A * exp(-(x * x) / (2.0 * w * w));",
                       "return A * exp(-(x * x) / (w * w));"),
    "pulse_width_power": ("pins", "dh[2] = A * e * x * x / (w * w * w);",
                          "dh[2] = A * e * x * x / (w * w);"),
    "pulse_centre_sign": ("pins", "dh[1] = A * e * x / (w * w);", "dh[1] = -A * e * x / (w * w);"),
    "sine_chirp_factor": ("pins", "PI * fdot * t * t + phi0;\n    return A * sin(phase);",
                          "TWO_PI * fdot * t * t + phi0;\n    return A * sin(phase);"),
    "sine_frequency_derivative": ("pins", "dh[1] = TWO_PI * t * A * c;", "dh[1] = TWO_PI * A * c;"),
    "residual_skip_index": ("pins", "if (k != skip) hs += template_value(model, th + k * P, t);",
                            "if (k > skip) hs += template_value(model, th + k * P, t);"),
    "logl_sigma_squared": ("pins", "1.0;\n    logl[i] = b * (-0.5 * ss / (sigma * sigma));",
                           "1.0;\n    logl[i] = b * (-0.5 * ss / sigma);"),
    "gradient_tempering": ("pins", "g[k] = b * (g[k] / (sigma * sigma));\n    if (logl)",
                           "g[k] = g[k] / (sigma * sigma);\n    if (logl)"),
    "birth_energy_factor": ("pins", "d_birth[i] = b * (x - 0.5 * y) / (sigma * sigma);",
                            "d_birth[i] = b * (x - y) / (sigma * sigma);"),
    "death_sign": ("pins", "d_death[i] = -(b * (x - 0.5 * y) / (sigma * sigma));",
                   "d_death[i] = -(b * (x + 0.5 * y) / (sigma * sigma));"),
    "segment_start": ("pins", "for (int64_t s = T1; s < T2; ++s) {", "for (int64_t s = T1 + 1; s < T2; ++s) {"),
    "logsumexp_shift": ("pins", "scalars[1] = m + log(s1) - lse_prev;", "scalars[1] = log(s1) - lse_prev;"),
    "ess_square": ("pins", "scalars[0] = s1 * s1 / s2;", "scalars[0] = s1 / s2;"),
    "leapfrog_half_kick": ("pins", "double ph = p[m] + 0.5 * eps * grad_out[m];",
                           "double ph = p[m] + eps * grad_out[m];"),
    "leapfrog_drift": ("pins", "q_out[m] = q[m] + eps * ph;", "q_out[m] = q[m] + eps * p[m];"),
    # ---------------------------------------------------------------- metric
    "fisher_outer_product": ("metric", "Fi[a * n + c] += ws * (J[a] * J[c]);",
                             "Fi[a * n + c] += ws * (J[a] * J[a]);"),
    "fisher_tempering": ("metric", "double outer = split == 0 ? b : 1.0;", "double outer = 1.0;"),
    "ridge_parameter": ("metric", "double v = Fi[r * n + c] + (r == c ? ridge[r % P] : 0.0);",
                        "double v = Fi[r * n + c] + (r == c ? ridge[(r + 1) % P] : 0.0);"),
    "cholesky_short_sum": ("metric", "for (int64_t k = 0; k < c; ++k) v -= L[r * n + k] * L[c * n + k];",
                           "for (int64_t k = 1; k < c; ++k) v -= L[r * n + k] * L[c * n + k];"),
    "pivot_test": ("metric", "if (!(v > 0.0)) { ok = 0; break; }", "if (!(v > -1e300)) { ok = 0; break; }"),
    "substitution_index": ("metric", "for (int64_t k = c; k < r; ++k) v -= L[r * n + k] * Wi[k * n + c];",
                           "for (int64_t k = c + 1; k < r; ++k) v -= L[r * n + k] * Wi[k * n + c];"),
    "kick_wrong_side": ("metric", "matvec(Wi, n, 0, gF, wv);\n            for (int64_t x = 0; x < n; ++x) pF[x] = pF[x] + 0.5 * e * wv[x];",
                        "matvec(Wi, n, 1, gF, wv);\n            for (int64_t x = 0; x < n; ++x) pF[x] = pF[x] + 0.5 * e * wv[x];"),
    "drift_wrong_side": ("metric", "matvec(Wi, n, 1, pF, wv);", "matvec(Wi, n, 0, pF, wv);"),
    "fisher_split_weight": ("metric", "double ws = split == 0 ? 1.0 : sample_weight(s, split, b);",
                            "double ws = split == 0 ? 1.0 : b;"),
    # ---------------------------------------------------------------- frequency-domain GB
    "channel_A_coefficient": ("gb", "DA9[3 * i + j] = (M[2][i][j] - M[0][i][j]) / sqrt(2.0);",
                              "DA9[3 * i + j] = (M[2][i][j] - M[0][i][j]) / sqrt(3.0);"),
    "plus_tensor_sign": ("gb", "ep[i][j] = u[i] * u[j] - v[i] * v[j];", "ep[i][j] = u[i] * u[j] + v[i] * v[j];"),
    "psi_rotation": ("gb", "Fp[c] = cos(2.0 * psi) * P + sin(2.0 * psi) * X;",
                     "Fp[c] = cos(psi) * P + sin(psi) * X;"),
    "doppler_sign": ("gb", "double tau = t + kAU * cos(b) * cos(a - l) / kC;",
                     "double tau = t - kAU * cos(b) * cos(a - l) / kC;"),
    "orbit_phase": ("gb", "double a = 2.0 * kPi * t / kYear;\n  double e = kArm",
                    "double a = kPi * t / kYear;\n  double e = kArm"),
    "window_placement": ("gb", "int64_t k = q + m - k0;", "int64_t k = q + m - k0 + 1;"),
    "dft_scale": ("gb", "double scale = T_obs / (double)Ns;", "double scale = T_obs / (double)(Ns - 1);"),
    "envelope_sign": ("gb", "z[c][1] = 0.5 * (ar * sph + ai * cph);", "z[c][1] = 0.5 * (ar * sph - ai * cph);"),
    "fdot_phase_derivative": ("gb", "dphi[1] = kPi * tau * tau;", "dphi[1] = 2.0 * kPi * tau * tau;"),
    "longitude_phase_derivative": ("gb", "dphi[4] = 2.0 * kPi * fi * (kAU * cos(b) * sin(a - l) / kC);",
                                   "dphi[4] = 2.0 * kPi * fi * (kAU * cos(b) * cos(a - l) / kC);"),
    "psi_amplitude_derivative": ("gb", "da[5][0] = 2.0 * Fx[c] * Ap;", "da[5][0] = Fx[c] * Ap;"),
    "inclination_derivative_sign": ("gb", "da[6][1] = -Fx[c] * (2.0 * A * si);", "da[6][1] = Fx[c] * (2.0 * A * si);"),
    "gb_likelihood_normalisation": ("gb", "logl[i] = b * (-0.5 * cnorm * ss);", "logl[i] = b * (-cnorm * ss);"),
    "gb_death_sign": ("gb", "d_death[i] = -(b * cnorm * (rh + 0.5 * hh));", "d_death[i] = -(b * cnorm * (rh - 0.5 * hh));"),
    "gb_metric_channel_sum": ("gb", "for (int64_t x = 0; x < 4 * B; ++x) s += dh[pa * 4 * B + x] * dh[pb * 4 * B + x];",
                              "for (int64_t x = 0; x < 2 * B; ++x) s += dh[pa * 4 * B + x] * dh[pb * 4 * B + x];"),
    "gb_metric_tempering": ("gb", "Fi[(k * GB_P + pa) * n + k * GB_P + pb] = b * cnorm * s;",
                            "Fi[(k * GB_P + pa) * n + k * GB_P + pb] = cnorm * s;"),
    "gb_metric_block_placement": ("gb", "Fi[(k * GB_P + pa) * n + k * GB_P + pb] = b * cnorm * s;",
                                  "Fi[(k * GB_P + pa) * n + pb] = b * cnorm * s;"),
    # ---------------------------------------------------------------- SMC steps
    "ess_ratio": ("smc", "return s1 * s1 / s2;", "return s1 / s2;"),
    "ess_weight_square": ("smc", "double e = exp(lw - m);\n    s1 += e;\n    s2 += e * e;",
                          "double e = exp(lw - m);\n    s1 += e;\n    s2 += e;"),
    "tempering_increment": ("smc", "logw[i] = (logw_prev ? logw_prev[i] : 0.0) + db * logl[i];",
                            "logw[i] = (logw_prev ? logw_prev[i] : 0.0) + beta * logl[i];"),
    "bisection_side": ("smc", "if (e >= target) {\n        lo = mid;", "if (e < target) {\n        lo = mid;"),
    "full_step_test": ("smc", "ess_at(N, logl, logw_prev, 1.0 - beta_prev, NULL, NULL)",
                       "ess_at(N, logl, logw_prev, 1.0, NULL, NULL)"),
    "evidence_uniform_normaliser": ("smc", "    lse_prev = log((double)N);\n  }\n  scalars[0] = beta;",
                                    "    lse_prev = 0.0;\n  }\n  scalars[0] = beta;"),
    "evidence_shift": ("smc", "scalars[2] = m + log(s1) - lse_prev;", "scalars[2] = log(s1) - lse_prev;"),
    "resample_offset": ("smc", "floor(((double)j + u) * (double)total / (double)N)",
                        "floor(((double)j + 0.5) * (double)total / (double)N)"),
    "resample_search": ("smc", "while (C[a] <= U) ++a;", "while (C[a] < U) ++a;"),
    "resample_copy_source": ("smc", "theta_out[offsets_out[j] * P + x] = theta[offsets[a] * P + x];",
                             "theta_out[offsets_out[j] * P + x] = theta[offsets[j] * P + x];"),
    "birth_ratio_sign": ("smc", "acc = log_u[i] < dlogl_birth[i] + log_pd_over_pb;",
                         "acc = log_u[i] < dlogl_birth[i] - log_pd_over_pb;"),
    "death_ratio_sign": ("smc", "acc = log_u[i] < dlogl_death[i] - log_pd_over_pb;",
                         "acc = log_u[i] < dlogl_death[i] + log_pd_over_pb;"),
    "birth_k_bound": ("smc", "K + 1 <= k_hi", "K + 1 < k_hi"),
    "death_row_removed": ("smc", "if (k == skip) continue;", "if (k == skip + 1) continue;"),
    # ---------------------------------------------------------------- posterior-start bridge
    "split_boundary": ("split", "return s < split ? 1.0 : b;", "return s <= split ? 1.0 : b;"),
    "split_swapped_weights": ("split", "return s < split ? 1.0 : b;", "return s < split ? b : 1.0;"),
    "split_logl_unweighted": ("split", "ss += sample_weight(s, split, b) * (r * r);", "ss += r * r;"),
    "split_gradient_unweighted": ("split", "for (int p = 0; p < P; ++p) g[k * P + p] += ws * (r * dh[p]);",
                                  "for (int p = 0; p < P; ++p) g[k * P + p] += r * dh[p];"),
    "split_birth_energy_unweighted": ("split", "        x += ws * (r * h);\n        y += ws * (h * h);\n      }\n      d_birth[i]",
                                      "        x += ws * (r * h);\n        y += h * h;\n      }\n      d_birth[i]"),
    "split_death_energy_sign": ("split", "d_death[i] = -((x - 0.5 * y) / (sigma * sigma));",
                                "d_death[i] = -((x + 0.5 * y) / (sigma * sigma));"),
    "split_nuts_wrong_target": ("split", "particle_logl_grad_split(model, d, T, t_start, dt, sigma, K, qF, b, split, &lF, gF);",
                                "particle_logl_grad(model, d, T, t_start, dt, sigma, K, qF, b, &lF, gF);"),
}

# the pins that take longest run last: most mutants fail a fast one first
_SLOW = ("brute_force", "dft", "aliasing", "sky_averaged")


def _calls(group):
    """(name, function, keyword arguments) of every CPU pin of a group, with
    pytest's parametrize marks expanded."""
    out = []
    for modname in GROUPS[group]:
        mod = importlib.import_module(modname)
        for name, fn in inspect.getmembers(mod, inspect.isfunction):
            if not name.startswith("test_") or fn.__module__ != mod.__name__:
                continue
            marks = getattr(fn, "pytestmark", [])
            if any(m.name in ("gpu", "skip") for m in marks):
                continue
            combos = [{}]
            for m in marks:
                if m.name != "parametrize":
                    continue
                names = [x.strip() for x in m.args[0].split(",")]
                new = []
                for c in combos:
                    for v in m.args[1]:
                        vals = getattr(v, "values", None)
                        if vals is None:
                            vals = tuple(v) if len(names) > 1 else (v,)
                        new.append({**c, **dict(zip(names, vals))})
                combos = new
            for c in combos:
                out.append((f"{modname}::{name}{c if c else ''}", fn, c))
    out.sort(key=lambda x: any(k in x[0] for k in _SLOW))
    return out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(orc, tmp_path, monkeypatch, name):
    group, old, new = MUTANTS[name]
    path = orc.build_variant(str(tmp_path), [(old, new)])
    monkeypatch.setattr(orc, "_lib", orc.bind(path))
    for label, fn, kw in _calls(group):
        args = {"orc": orc, **kw}
        if "tmp_path" in inspect.signature(fn).parameters:
            args["tmp_path"] = tmp_path
        try:
            fn(**args)
        except Exception:  # noqa: BLE001 - any failing pin catches the mistake
            return
    pytest.fail(f"planted mistake {name} passed every pin of group {group}")
