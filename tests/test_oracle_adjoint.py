"""The oracle's adjoint step against the forward oracle (CPU only)."""
import pytest

import adjoint_pins
import oracle


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("check", adjoint_pins.FAST_ADJOINT_CHECKS, ids=lambda f: f.__name__)
def test_adjoint_pin(orc, check):
    check(orc)
