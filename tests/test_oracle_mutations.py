"""Plant plausible mistakes in the oracle (on the CPU, via monkeypatch) and
check that the pins catch each one: a pin that passes a wrong oracle pins
nothing."""
import numpy as np
import pytest

from oracle import moments, sweep
import tests.test_oracle_moments as tm
import tests.test_oracle_sweep as ts


def _segment_step_wrong_source(I, kappa_t, Q, length, sin_zeta):
    # mistake: the source divided by kappa instead of the modified opacity
    tau = kappa_t * length / sin_zeta
    e = np.exp(-tau)
    src = Q / (kappa_t - 1.0 / 3.0)
    I_out = I * e + src * (-np.expm1(-tau))
    a = sweep.alpha_of_tau(tau)
    return I_out, a * I + (1 - a) * I_out


def _segment_step_swapped_alpha(I, kappa_t, Q, length, sin_zeta):
    # mistake: alpha weights the outgoing intensity instead of the incoming one
    tau = kappa_t * length / sin_zeta
    I_out = I * np.exp(-tau) + Q / kappa_t * (-np.expm1(-tau))
    a = sweep.alpha_of_tau(tau)
    return I_out, (1 - a) * I + a * I_out


def _segment_step_no_sin(I, kappa_t, Q, length, sin_zeta):
    # mistake: in-plane length used as the path length
    return _orig_step(I, kappa_t, Q, length, 1.0)


_orig_step = sweep.segment_step


@pytest.mark.parametrize("bad", [_segment_step_wrong_source, _segment_step_swapped_alpha,
                                 _segment_step_no_sin])
def test_segment_mistakes_are_caught(monkeypatch, bad):
    monkeypatch.setattr(sweep, "segment_step", bad)
    caught = 0
    for pin in (ts.test_uniform_absorber_exit_and_segment_averages,
                lambda: ts.test_tiny_grid_against_ode_integration(2, 2)):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1


def test_direction_mapping_mistake_is_caught(monkeypatch):
    # mistake: the reverse traversal mapped onto the forward azimuth
    monkeypatch.setattr(sweep, "direction_index",
                        lambda a, d, p, n_az, n_pol: a * n_pol + p)
    monkeypatch.setattr(moments, "direction_index",
                        lambda a, d, p, n_az, n_pol: a * n_pol + p)
    with pytest.raises(AssertionError):
        tm.test_single_direction_indicator_cells()


def test_alpha_sign_mistake_is_caught(monkeypatch):
    orig = sweep.alpha_of_tau
    monkeypatch.setattr(sweep, "alpha_of_tau", lambda t: 1.0 - orig(t))
    with pytest.raises(AssertionError):
        ts.test_alpha_matches_high_precision()
    with pytest.raises(AssertionError):
        ts.test_uniform_absorber_exit_and_segment_averages()
