"""Plant plausible mistakes in copies of the oracle and check that a pin catches each.

Each mutant is a textual change of ``oracle/lv_oracle.c`` compiled into a
temporary library; the pins of tests/pins.py run against it in order of cost and
at least one must fail.  This shows that the pins constrain every step of the
oracle: stepping, random numbers, interpolation, payoffs and the reverse sweep.
"""
import os
import tempfile

import pytest

import oracle
from tests import pins

MUTANTS = {
    "drift_dropped": ("w->y[n] + (pb->rate - 0.5 * s * s) * dt + s * sdt * w->z[n]", "w->y[n] + pb->rate * dt + s * sdt * w->z[n]"),
    "sqrt_dt_wrong": ("pb->sqrt_dt = sqrt(pb->dt);", "pb->sqrt_dt = pb->dt;"),
    "box_muller_sin_cos_swapped": ("if (r % 2 == 0)\n        return radius * cos", "if (r % 2 == 1)\n        return radius * cos"),
    "uniform_not_centred": ("+ 0.5) / 8388608.0", "+ 0.0) / 8388608.0"),
    "philox_weyl_constant": ("k0 += PHILOX_W0;", "k0 += PHILOX_W1;"),
    "philox_nine_rounds": ("round < 10", "round < 9"),
    "weights_transposed": ("out->w[1] = (1.0 - alpha) * f;\n    out->w[2] = alpha * (1.0 - f);",
                           "out->w[1] = alpha * (1.0 - f);\n    out->w[2] = (1.0 - alpha) * f;"),
    "time_weight_flipped": ("*alpha = b - jj;", "*alpha = 1.0 - (b - jj);"),
    "spot_not_clamped_above": ("if (a > pb->n_spot - 1) a = pb->n_spot - 1;", ""),
    "slope_times_du": ("alpha * (s11 - s01)) / du;", "alpha * (s11 - s01)) * du;"),
    "log_axis_chain_rule": ("(pb->spot_kind == 0) ? dsdu * S : dsdu", "dsdu * S"),
    "sigma_at_right_point": ("lvo_eval(pb, S, n * dt, &w->iv[n]);", "lvo_eval(pb, S, (n + 1) * dt, &w->iv[n]);"),
    "adjoint_c_sign": ("double c = -iv->sigma * dt + sdt * w->z[n - 1];", "double c = iv->sigma * dt + sdt * w->z[n - 1];"),
    "adjoint_no_spot_slope": ("lam = lam * (1.0 + c * iv->dsigma_dy);", "lam = lam * 1.0;"),
    "adjoint_wrong_node": ("grad[iv->i * J + iv->j + 1] += gbar * iv->w[2];", "grad[(iv->i + 1) * J + iv->j + 1] += gbar * iv->w[2];"),
    "put_derivative_sign": ("if (pb->is_put[k]) return K > S ? -S : 0.0;", "if (pb->is_put[k]) return K > S ? S : 0.0;"),
    "payoff_at_last_step": ("payoffs[k] = pb->disc[k] * lvo_payoff(pb, k, w->y[pb->tap_step[k]]);", "payoffs[k] = pb->disc[k] * lvo_payoff(pb, k, w->y[N]);"),
    "cotangent_weight_ignored": ("double wk = pb->weight ? pb->weight[k] : 1.0;", "double wk = 1.0;"),
    "euler_x_lognormal_step": ("X[n + 1] = X[n] + pb->rate * X[n] * dt + w->iv[n].sigma * X[n] * sdt * w->z[n];",
                               "X[n + 1] = X[n] * exp(w->iv[n].sigma * sdt * w->z[n] - 0.5 * w->iv[n].sigma * w->iv[n].sigma * dt);"),
    "euler_x_c_without_X": ("double c = X[n - 1] * sdt * w->z[n - 1];", "double c = sdt * w->z[n - 1];"),
    "euler_x_no_spot_slope": ("(iv->sigma + iv->dsigma_dy)", "(iv->sigma)"),
    "euler_x_wrong_node": ("grad[q00 + 1] += lam * c * iv->w[2];", "grad[q00 + J + 1] += lam * c * iv->w[2];"),
    "bf16_truncates": ("if (d_lo < d_hi) pick = below;", "if (1) pick = below;"),
    "bf16_ties_away": ("else pick = (below & 0x10000u) ? above : below;", "else pick = above;"),
    "bf16_ties_odd": ("else pick = (below & 0x10000u) ? above : below;", "else pick = (below & 0x10000u) ? below : above;"),
    "bf16_straight_from_double": ("const double x = (double)lvo_bits_to_float(mag);", "const double x = fabs(v);"),
    "rate_drift_sign": ("(pb->rate - 0.5 * s * s) * dt", "(-pb->rate - 0.5 * s * s) * dt"),
    "rate_in_the_diffusion": ("(pb->rate - 0.5 * s * s) * dt + s * sdt * w->z[n]", "(-0.5 * s * s) * dt + (s + pb->rate) * sdt * w->z[n]"),
    "rate_not_discounted": ("pb->disc[k] = exp(-pb->rate * pb->maturity[k]);", "pb->disc[k] = 1.0;"),
    "rate_discount_at_last_maturity": ("pb->disc[k] = exp(-pb->rate * pb->maturity[k]);", "pb->disc[k] = exp(-pb->rate * pb->dt * pb->n_steps);"),
    "rate_seed_undiscounted": ("lam += wk * pb->disc[k] * lvo_dpayoff_dy(pb, k, w->y[n]);", "lam += wk * lvo_dpayoff_dy(pb, k, w->y[n]);"),
    "rate_euler_x_trend_missing": ("X[n + 1] = X[n] + pb->rate * X[n] * dt + w->iv[n].sigma", "X[n + 1] = X[n] + w->iv[n].sigma"),
    "rate_euler_x_jacobian_without_trend": ("lam * (1.0 + pb->rate * dt + sdt", "lam * (1.0 + sdt"),
}

BATTERY = [pins.pin_round_bf16, pins.pin_uniform, pins.pin_box_muller, pins.pin_interp, pins.pin_flat_pathwise_vega,
           pins.pin_one_step, pins.pin_adjoint_fd, pins.pin_put_call_parity,
           pins.pin_flat_black_scholes, pins.pin_term_structure, pins.pin_euler_x_one_step,
           pins.pin_euler_x_moments, pins.pin_rate_adjoint_fd, pins.pin_rate_parity_and_martingale,
           pins.pin_rate_one_step, pins.pin_rate_euler_x_one_step, pins.pin_rate_black_scholes]


def _build_mutant(name, old, new, tmpdir):
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/present"
    path = os.path.join(tmpdir, f"{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    return oracle.build(path, os.path.join(tmpdir, f"lib_{name}.so"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    lib = _build_mutant(name, old, new, str(tmp_path))
    mutant = oracle.Oracle(lib)
    battery = list(BATTERY)
    if pins.rocrand_available():
        battery.insert(0, pins.pin_philox_rocrand)
    caught = []
    for pin in battery:
        try:
            pin(mutant)
        except (AssertionError, oracle.OracleError, FloatingPointError, ValueError) as e:
            caught.append((pin.__name__, str(e)[:120]))
            break
    assert caught, f"no pin caught mutant {name}"
