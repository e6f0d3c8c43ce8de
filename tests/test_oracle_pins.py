"""The CPU oracle against the facts that pin it (see tests/pins.py)."""
import pytest

import oracle
from tests import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.skipif(not pins.rocrand_available(), reason="hipcc / rocRAND headers not present")
def test_philox_matches_rocrand(orc):
    pins.pin_philox_rocrand(orc)


@pytest.mark.parametrize("pin", [
    pins.pin_uniform, pins.pin_box_muller, pins.pin_interp, pins.pin_flat_black_scholes,
    pins.pin_flat_pathwise_vega, pins.pin_flat_vega_and_columns, pins.pin_term_structure,
    pins.pin_put_call_parity, pins.pin_threads, pins.pin_one_step, pins.pin_two_steps,
    pins.pin_adjoint_fd, pins.pin_zero_buckets, pins.pin_euler_x_one_step, pins.pin_euler_x_moments,
    pins.pin_round_bf16, pins.pin_rate_black_scholes, pins.pin_rate_parity_and_martingale,
    pins.pin_rate_one_step, pins.pin_rate_euler_x_one_step, pins.pin_rate_adjoint_fd,
], ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_rejects_bad_inputs(orc):
    import numpy as np
    import workloads as W
    s = W.small_surface()
    with pytest.raises(oracle.OracleError):
        orc.price_and_grad(s, W.call(100.0, 1.0), 64, 52, want_grad=False, spot=-1.0)
    with pytest.raises(oracle.OracleError):      # 0.3y is not a whole number of 1/52 steps
        orc.price_and_grad(s, W.Book([0, 0], [100.0, 100.0], [1.0, 0.3], [1, 1]), 64, 52)
    bad = W.Surface(s.spot_axis, s.time_axis, np.where(np.arange(s.sigma.size).reshape(s.sigma.shape) == 5, np.nan, s.sigma))
    with pytest.raises(oracle.OracleError):
        orc.price_and_grad(bad, W.call(100.0, 1.0), 64, 52)
