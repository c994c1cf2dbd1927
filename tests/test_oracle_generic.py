"""The oracle's generic compartmental step (D2Q5 and D2Q9) against the SEIRD
oracle, closed forms, Fourier analysis and invariants (CPU only)."""
import pytest

import generic_pins
import oracle


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("check", generic_pins.FAST_GENERIC_CHECKS, ids=lambda f: f.__name__)
def test_generic_pin(orc, check):
    check(orc)


def test_d2q9_symbol_reading():
    generic_pins.check_d2q9_symbol_reading()
