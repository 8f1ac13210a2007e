"""The CPU oracle against what the paper and mathematics fix (see tests/_pins.py for the sources)."""
import pytest

import _pins


@pytest.mark.parametrize("name", _pins.curve_fixture_names())
def test_golden_curves(name):
    _pins.pin_golden(name=name)


def test_threshold_rule():
    _pins.pin_threshold_rule()


def test_closed_form_totals():
    _pins.pin_closed_form_totals()


def test_special_cases():
    _pins.pin_special_cases()


def test_symmetries():
    _pins.pin_symmetries()


def test_bounds():
    _pins.pin_bounds()


def test_half_neighbourhood_alg1():
    _pins.pin_alg1()


def test_direct_dilation_route():
    _pins.pin_direct_dilation()


def test_other_neighbourhoods_golden():
    _pins.pin_nbhd_golden()


def test_other_neighbourhoods_alg1():
    _pins.pin_nbhd_alg1()


def test_other_neighbourhoods_closed_forms():
    _pins.pin_nbhd_closed_forms()


def test_other_neighbourhoods_reductions():
    _pins.pin_nbhd_reductions()


def test_other_neighbourhoods_direct():
    _pins.pin_nbhd_direct()


def test_binomial_prefilter():
    _pins.pin_binomial3()


def test_same_double_fixture_is_meaningful():
    """The exact-compare fixture only tests something if the two values collide as doubles."""
    from fractions import Fraction
    a, b = Fraction(1, 3), Fraction(333333333333333334, 10**18)
    assert a < b and float(a) == float(b)


def test_segment_pins():
    _pins.pin_segment()


def test_class_stats_pins():
    _pins.pin_class_stats()
