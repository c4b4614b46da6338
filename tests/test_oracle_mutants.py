"""The oracle's pins are sharp: plant one plausible mistake at a time in a copy of the
oracle source (on the CPU), rebuild it, and check that the pin suite fails on it."""
import inspect
import os

import pytest

import oracle
import test_oracle_pins as pins

# (name, original text, planted mistake) -- each original must occur in fcn_oracle.c
MUTANTS = [
    ("printed_cj_fj_factor", "double hi = 1.0 + 1.0 / (2.0 * j);", "double hi = 1.0 - 1.0 / (2.0 * j);"),
    ("axis_row_weight", "b[0] = 1.0 + I * diff * dz / kdr2", "b[0] = 1.0 + I * diff * dz / (2.0 * kdr2)"),
    ("gvd_sign", "b[j] = 1.0 + I * diff * dz / (2.0 * kdr2) - I * gvd;",
     "b[j] = 1.0 + I * diff * dz / (2.0 * kdr2) + I * gvd;"),
    ("omega_index", "int q = (p < nt / 2) ? p : p - nt;", "int q = p;"),
    ("rhs_lower_index", "if (j > 0) s += d[j] * col[j - 1];", "if (j > 0) s += d[j] * col[j];"),
    ("thomas_back_sign", "x[j] = dp[j] - cp[j] * x[j + 1];", "x[j] = dp[j] + cp[j] * x[j + 1];"),
    ("inverse_scale", "for (int i = 0; i < n; i++) x[i] *= s;", "for (int i = 0; i < n; i++) x[i] *= 1.0;"),
    ("twiddle_conj", "if (inverse) w = conj(w);", "if (!inverse) w = conj(w);"),
    ("rk4_weight", "k1 + 2.0 * k2 + 2.0 * k3 + k4", "k1 + 2.0 * k2 + k3 + k4"),
    ("rk4_midpoint", "ih = 0.5 * (i0 + i1);", "ih = i0;"),
    ("rate_saturation", "* (1.0 - rho / pp->rho_at);", ";"),
    ("plasma_sign", "nhat += -I * (dv->k0 / 2.0) * (rho / dv->rho_c);", "nhat += I * (dv->k0 / 2.0) * (rho / dv->rho_c);"),
    ("mpa_power", "pow(inten, (double)(pp->K - 1))", "pow(inten, (double)(pp->K))"),
    ("kerr_n4_dropped", "pp->n4 * inten * inten", "0.0 * inten * inten"),
    ("half_step_length", "if (orc_nl_half(pp, field, 0.5 * dz, nthreads)) return 1;",
     "if (orc_nl_half(pp, field, dz, nthreads)) return 1;"),
    ("energy_axis_weight", "double e = 0.125 * rowsum[0];", "double e = 0.25 * rowsum[0];"),
    ("adaptive_lag", "double phi_lag = (n == 0) ? diag[4] : phi_prev;", "double phi_lag = diag[4];"),
    ("coll_sign", "nhat += -(pp->sigma_c / 2.0) * rho;", "nhat += (pp->sigma_c / 2.0) * rho;"),
    ("coll_half_dropped", "nhat += -(pp->sigma_c / 2.0) * rho;", "nhat += -pp->sigma_c * rho;"),
    ("kerr_n6_dropped", "pp->n6 * pow(inten, 3.0)", "0.0 * pow(inten, 3.0)"),
    ("kerr_n8_dropped", "pp->n8 * pow(inten, 4.0)", "0.0 * pow(inten, 4.0)"),
    ("kerr_n6_power", "pp->n6 * pow(inten, 3.0)", "pp->n6 * pow(inten, 2.0)"),
    ("mpa_half_dropped", "nhat += -(dv->betaK / 2.0) * pow(", "nhat += -(dv->betaK) * pow("),
    ("avalanche_sign", "r += pp->sigma_c / pp->U_i * intensity * rho;", "r -= pp->sigma_c / pp->U_i * intensity * rho;"),
    ("avalanche_no_intensity", "r += pp->sigma_c / pp->U_i * intensity * rho;", "r += pp->sigma_c / pp->U_i * rho;"),
    ("avalanche_saturated", "r += pp->sigma_c / pp->U_i * intensity * rho;",
     "r += pp->sigma_c / pp->U_i * intensity * rho * (1.0 - rho / pp->rho_at);"),
]


def _pin_tests():
    out = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        if params:
            argname, values = params[0].args
            for v in values:
                out.append((f"{name}[{v}]", fn, {argname: v}))
        else:
            out.append((name, fn, {}))
    return out


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, orig, bad):
    src = oracle.source()
    assert src.count(orig) >= 1, f"mutation site for {name} not found"
    path = oracle.compile_variant(src.replace(orig, bad, 1), os.path.join(tmp_path, f"lib_{name}.so"))
    caught = []
    with oracle.use_library(path):
        for tname, fn, kw in _pin_tests():
            try:
                if "orc" in inspect.signature(fn).parameters:
                    fn(orc=oracle, **kw)
                else:
                    fn(**kw)
            except Exception:  # an assertion, or a non-finite result that numpy trips on
                caught.append(tname)
                break
    assert caught, f"no pin fails on mutant {name}"
